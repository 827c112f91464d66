// Decoupled look-back by one wavefront, 64 predecessors per round.
#pragma once

#include "capt_internal.h"

namespace capt {

// Exclusive prefix of tile t from the words its predecessors publish in
// status[]: bits 30-31 = 1 (the tile's own sum) or 2 (its inclusive prefix),
// bits 0-29 = the value, 0 while nothing is published.  All 64 lanes of one
// wavefront call it together: in a round lane i reads tile t - 1 - i (waiting
// until it is published), the wave adds the values from the nearest inclusive
// prefix on and stops there, else goes 64 tiles further back.  A tile waits
// only for tiles with smaller ids, which started before it; a wait longer than
// `spins` reads sets `errbit` in *err and stops the walk.
__device__ inline uint32_t wave_lookback(const uint32_t *status, int64_t t, uint32_t spins, uint32_t *err,
                                         uint32_t errbit) {
    const int lane = threadIdx.x & (WAVE - 1);
    uint32_t excl = 0;
    for (int64_t hi = t; hi > 0; hi -= WAVE) {
        const int64_t q = hi - 1 - lane;
        uint32_t v = 2u << 30;   // lanes before tile 0: an empty inclusive prefix
        if (q >= 0) {
            uint32_t n = 0;
            while (((v = __hip_atomic_load(&status[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 30) == 0u) {
                if (++n > spins) {
                    atomicOr(err, errbit);
                    v = 2u << 30;
                    break;
                }
            }
        }
        const uint64_t pre = __ballot((v >> 30) == 2u);
        const int stop = pre ? __builtin_ctzll(pre) : WAVE;   // the nearest inclusive prefix
        uint32_t c = lane <= stop ? (v & ((1u << 30) - 1u)) : 0u;
        for (int off = WAVE / 2; off >= 1; off >>= 1) c += (uint32_t)__shfl_xor((int)c, off, WAVE);
        excl += c;
        if (pre) break;
    }
    return excl;
}

}  // namespace capt
