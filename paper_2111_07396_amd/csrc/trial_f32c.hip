// Trial kernels of the compensated-FP32 policy (templates in trial_impl.hpp).
#include "trial_impl.hpp"

namespace ssg {

hipError_t launch_trials_f32c(int shape, const TrialLaunch &L, int64_t max_items, int n_cu,
                              hipStream_t s) {
    return launch_policy<F32C>(shape, L, max_items, n_cu, s);
}

}  // namespace ssg
