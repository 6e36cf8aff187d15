// Trial kernels of the FP64 policy, the launch dispatch over precisions, and
// the host-side layout helpers.  The kernels are templates in trial_impl.hpp.
#include "trial_impl.hpp"

namespace ssg {

hipError_t launch_trials_f32c(int shape, const TrialLaunch &L, int64_t max_items, int n_cu,
                              hipStream_t s);

int trial_lds_bytes(int nw, int ppl, int ext, int method) {
    return Layout(nw, ppl, ext, method).bytes;
}

int trial_halfwidth(int n, double span) { return halfwidth(n, span); }

hipError_t launch_checks(int shape, const TrialLaunch &L, int64_t max_items, int n_cu,
                         unsigned long long *counts, int selftest, hipStream_t s) {
    return launch_checks_shape(shape, L, max_items, n_cu, counts, selftest, s);
}

hipError_t launch_trials(int shape, int precision, const TrialLaunch &L, int64_t max_items,
                         int n_cu, hipStream_t s) {
    return precision == 0 ? launch_policy<F64>(shape, L, max_items, n_cu, s)
                          : launch_trials_f32c(shape, L, max_items, n_cu, s);
}

}  // namespace ssg
