// ssp_df.h - complex FP32 arithmetic shared by the device kernels: plain complex products and
// products with a double-float (hi + lo) complex factor.
#pragma once

#include <hip/hip_runtime.h>

namespace ssp {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// x * (w.hi + w.lo) with w = (hi.re, hi.im, lo.re, lo.im): the small products first, so the
// result carries only the rounding of the arithmetic, not the rounding of the table.
__device__ __forceinline__ float2 cmul_df(float2 x, float4 w) {
    float re = fmaf(-x.y, w.w, x.x * w.z);
    re = fmaf(x.x, w.x, re);
    re = fmaf(-x.y, w.y, re);
    float im = fmaf(x.y, w.z, x.x * w.w);
    im = fmaf(x.x, w.y, im);
    im = fmaf(x.y, w.x, im);
    return make_float2(re, im);
}
// x * conj(w.hi + w.lo)
__device__ __forceinline__ float2 cmul_df_conj(float2 x, float4 w) {
    float re = fmaf(x.y, w.w, x.x * w.z);
    re = fmaf(x.x, w.x, re);
    re = fmaf(x.y, w.y, re);
    float im = fmaf(-x.x, w.w, x.y * w.z);
    im = fmaf(-x.x, w.y, im);
    im = fmaf(x.y, w.x, im);
    return make_float2(re, im);
}
__device__ __forceinline__ float cnorm2(float2 v) { return fmaf(v.x, v.x, v.y * v.y); }

}  // namespace ssp
