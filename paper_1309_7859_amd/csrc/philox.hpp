// philox.hpp -- Philox4x32-10 counter-based generator (Salmon, Moraes, Dror
// and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) and the
// Gaussian displacements of the serving replicas drawn from it.
//
// Stream definition (a replica has a 64-bit seed, steps t = 0, 1, ..., ions i):
//   key = (seed & 0xffffffff, seed >> 32), counter = (i, t, j, 0) for j = 0, 1
//   each call gives words x0..x3; uniforms u = ((x_a >> 5) * 2^26 + (x_b >> 6)) / 2^53
//   from (x0, x1) and (x2, x3); Box-Muller: r = sqrt(-2 ln(1 - u_a)),
//   n_a = r cos(2 pi u_b), n_b = r sin(2 pi u_b)
//   call j = 0 gives the x and y normals, call j = 1 the z normal (its second
//   normal is unused); the displacement is sigma times the normal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace memd {

struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t p0 = (uint64_t)M0 * c0;
        const uint64_t p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    Philox4 r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

// Displacement of ion i at step t (three components).
__device__ __forceinline__ void philox_displacement(uint64_t seed, uint32_t t, uint32_t i, double sigma,
                                                    double (&du)[3]) {
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const double two_pi = 6.283185307179586476925286766559;
    const Philox4 a = philox4x32_10(i, t, 0u, 0u, k0, k1);
    const Philox4 b = philox4x32_10(i, t, 1u, 0u, k0, k1);
    double ua = u53(a.v[0], a.v[1]), ub = u53(a.v[2], a.v[3]);
    double rr = sqrt(-2.0 * log(1.0 - ua));
    du[0] = sigma * rr * cos(two_pi * ub);
    du[1] = sigma * rr * sin(two_pi * ub);
    ua = u53(b.v[0], b.v[1]);
    ub = u53(b.v[2], b.v[3]);
    rr = sqrt(-2.0 * log(1.0 - ua));
    du[2] = sigma * rr * cos(two_pi * ub);
}

// Component d of philox_displacement, with the same arithmetic (so that
// three lanes can draw one ion's three components side by side).
__device__ __forceinline__ double philox_displacement_component(uint64_t seed, uint32_t t, uint32_t i,
                                                                double sigma, int d) {
    const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
    const double two_pi = 6.283185307179586476925286766559;
    const Philox4 a = philox4x32_10(i, t, d == 2 ? 1u : 0u, 0u, k0, k1);
    const double ua = u53(a.v[0], a.v[1]), ub = u53(a.v[2], a.v[3]);
    const double rr = sqrt(-2.0 * log(1.0 - ua));
    return d == 1 ? sigma * rr * sin(two_pi * ub) : sigma * rr * cos(two_pi * ub);
}

}  // namespace memd
