// Learned lambda / stop-index model (filled in a later step).
#include "solve.h"

namespace abba {

int learned_prepare(const SolveDims &, const SolveWS &, const abba_reg *, hipStream_t) {
    set_error("the learned rule is not built yet");
    return ABBA_ERR_UNSUPPORTED;
}
int learned_features(const SolveDims &, const SolveWS &, hipStream_t) { return ABBA_ERR_UNSUPPORTED; }
int learned_judge(const SolveDims &, const SolveWS &, const abba_reg *, hipStream_t) { return ABBA_ERR_UNSUPPORTED; }

}  // namespace abba
