// device_util.hpp -- small device helpers: index wrapping, folding of unfolded
// coordinates, deterministic wavefront/block reductions (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace memd {

// Periodic wrap of i in [-L, inf) to [0, L).
__device__ __forceinline__ int wrapc(int i, int L) {
    if (i < 0) return i + L;
    if (i >= L) return i % L;
    return i;
}

// x / a, as an exponent shift when a is a power of two (then exactly the
// quotient), else a division.  a is the same for every lane, so the branch
// does not diverge; FP64 division is a long instruction sequence on the GPU.
__device__ __forceinline__ double div_a(double x, double a) {
    int e;
    const double m = frexp(a, &e);
    return m == 0.5 ? ldexp(x, 1 - e) : x / a;
}

// k mod L in [0, L) for an integer-valued double k with |k| < 2^51 L: the
// quotient's floor comes from k * (1/L), is off by at most one, and one
// correction fixes it; k - L q is then exact.  (No 64-bit integer division,
// which is a long software sequence on the GPU.)  The bound on |k| holds by
// construction: positions are rejected at entry beyond 2^40 box lengths and
// displacements beyond one box length per step.  The final clamp only keeps
// an index in bounds and never changes a result inside that range.
__device__ __forceinline__ int mod_cell(double k, int L) {
    const double Ld = (double)L;
    double m = k - Ld * floor(k * (1.0 / Ld));
    if (m < 0.0) m += Ld;
    else if (m >= Ld) m -= Ld;
    const int c = (int)m;
    return c < 0 ? 0 : (c >= L ? L - 1 : c);
}

// Fold an unfolded coordinate: t = u/a, k = floor(t), f = t - k in [0, 1),
// folded cell c = k mod L.
__device__ __forceinline__ void fold(double u, double a, int L, int &c, double &f) {
    const double t = div_a(u, a);
    const double fl = floor(t);
    f = t - fl;
    c = mod_cell(fl, L);
}

__device__ __forceinline__ double lin_w(int o, double f) { return o ? f : 1.0 - f; }

__device__ __forceinline__ size_t site_index(int i, int j, int k, int L) {
    return (size_t)i + (size_t)L * ((size_t)j + (size_t)L * (size_t)k);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Per-thread folds of W-vectors p[W b .. W b + W) over b = first, first +
// stride, ... < n, in increasing b (eight vectors' loads in flight per
// pass): column w is summed, or (bit w of maxmask) its maximum taken, from 0.
template <int W>
__device__ __forceinline__ void strided_fold(const double *__restrict__ p, int n, int first, int stride,
                                             unsigned maxmask, double (&s)[W]) {
#pragma unroll
    for (int w = 0; w < W; ++w) s[w] = 0.0;
    for (int b0 = first; b0 < n; b0 += 8 * stride) {
        double v[8][W];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * stride;
#pragma unroll
            for (int w = 0; w < W; ++w) v[u][w] = b < n ? p[W * b + w] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (b0 + u * stride < n) s[w] = ((maxmask >> w) & 1u) ? fmax(s[w], v[u][w]) : s[w] + v[u][w];
    }
}

template <int W>
__device__ __forceinline__ void strided_sum(const double *__restrict__ p, int n, int first, int stride,
                                            double (&s)[W]) {
    strided_fold<W>(p, n, first, stride, 0u, s);
}

// Block-wide sums of N values (blockDim.x a multiple of 64, <= 1024).  The
// result is returned to every thread; the summation order is fixed.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
    __shared__ double sh[N][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) sh[i][wid] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[i][w];
        v[i] = s;
    }
}

__device__ __forceinline__ double block_max(double v) {
    __shared__ double sh[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double m = sh[0];
    for (int w = 1; w < nw; ++w) m = fmax(m, sh[w]);
    return m;
}

// Map the hardware block id to a logical tile id so that consecutive logical
// tiles (spatial neighbours sharing halos) land on the same XCD: blocks are
// dealt round-robin over the 8 XCDs of an MI355X.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace memd
