// bw_launch.hpp -- internal interface between the C ABI layer and the
// Blackwell-family kernels (wm_blackwell.hip).
#pragma once

#include "bw_model.hpp"
#include "wm_launch.hpp"

namespace wm {

struct BwDescPtrs {
    const int32_t *bM, *bN, *bK, *G, *flags;
    const float *Kt, *CR, *ob;
};

hipError_t launch_bw_predict(const BwDescPtrs& d, int64_t n, const BwSet& S, float* T, int32_t* cta,
                             const LaunchCfg& cfg, hipStream_t s);
// mode 0: weights dL/dT, out = dL/dtheta[24]; mode 1: measured times, out =
// [loss, count, grad[24]]; S_dev != nullptr reads the set from device memory;
// out == nullptr skips the final reduction (rows: phase-1 blocks + nb2)
int bw_grad_grid(int mode, bool from_device_set, int64_t n, const LaunchCfg& cfg);
hipError_t launch_bw_grad(int mode, const BwDescPtrs& d, int64_t n, const float* w, const BwSet& S,
                          const BwSet* S_dev, double* partials, uint64_t* flags, const GradLayout& L,
                          const LaunchCfg& cfg, double* out, hipStream_t s);
hipError_t launch_bw_adam(const double* partials, int rows, CalibState* st, const AdamOpts& o,
                          BwSet* S, double* loss_hist, hipStream_t s);

}  // namespace wm
