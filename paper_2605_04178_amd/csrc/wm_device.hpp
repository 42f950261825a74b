// wm_device.hpp -- device-side helpers shared by the kernel files: streaming
// loads of one descriptor row and its float64 image.
#pragma once

#include "wm_launch.hpp"

namespace wm {

template <typename T>
__device__ inline T ntload(const T* p) { return __builtin_nontemporal_load(p); }

__device__ inline Desc<float> load_desc(const DescPtrs& d, int64_t i)
{
    Desc<float> x;
    x.F = ntload(d.F + i);
    x.B = ntload(d.B + i);
    x.r1 = ntload(d.r1 + i);
    x.r2 = ntload(d.r2 + i);
    x.r3 = ntload(d.r3 + i);
    x.K = ntload(d.K + i);
    x.u = ntload(d.u + i);
    x.W = ntload(d.W + i);
    x.v = ntload(d.vgpr + i);
    x.s = ntload(d.lds + i);
    x.gp = ntload(d.gpack + i);
    x.G = ntload(d.grid + i);
    return x;
}

__device__ inline Desc<double> widen(const Desc<float>& x)
{
    Desc<double> y;
    y.F = x.F; y.B = x.B; y.r1 = x.r1; y.r2 = x.r2; y.r3 = x.r3; y.K = x.K; y.u = x.u; y.W = x.W;
    y.v = x.v; y.s = x.s; y.gp = x.gp; y.G = x.G;
    return y;
}

}  // namespace wm
