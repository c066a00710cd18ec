// 3D circular cone-beam operators (filled in below in a later step).
#include "ops.h"

namespace abba {

int build_cone_tables(abba_op *op) {
    (void)op;
    set_error("cone-beam geometry is not built yet");
    return ABBA_ERR_UNSUPPORTED;
}

int cone_forward(const abba_op *, VecRef, VecRef, int, int, const Launch &) { return ABBA_ERR_UNSUPPORTED; }
int cone_back(const abba_op *, VecRef, int, VecRef, int, const Launch &) { return ABBA_ERR_UNSUPPORTED; }

}  // namespace abba
