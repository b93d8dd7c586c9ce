// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11) and Box-Muller
// normals, shared by the heat bath and the stochastic-estimation probes.
// Counter (element, index low word, purpose, index high word), key (seed low,
// seed high).  Purposes: 1 momenta, 2 pseudofermion source, 3 Metropolis
// uniform, 4 probe vectors (the index is then the measurement index).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace qh {

enum : uint32_t { RNG_MOMENTUM = 1, RNG_SOURCE = 2, RNG_METROPOLIS = 3, RNG_PROBE = 4 };

__device__ __forceinline__ void philox10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void draw_block(uint64_t seed, uint64_t traj, uint32_t purpose, uint32_t elem,
                                           uint32_t (&x)[4]) {
    x[0] = elem;
    x[1] = (uint32_t)traj;
    x[2] = purpose;
    x[3] = (uint32_t)(traj >> 32);
    philox10(x, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ void gauss_pair(const uint32_t (&x)[4], double& g1, double& g2) {
    const double u1 = uniform53(x[0], x[1]), u2 = uniform53(x[2], x[3]);
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    double s, c;
    sincos(2.0 * M_PI * u2, &s, &c);
    g1 = rad * c;
    g2 = rad * s;
}

}  // namespace qh
