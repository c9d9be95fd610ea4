// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11), host and device.
// Ten rounds of (hi0,lo0) = M0*x0, (hi1,lo1) = M1*x2, x <- (hi1^x1^k0, lo1, hi0^x3^k1, lo0), with
// the key advanced by the Weyl constants between rounds.
#pragma once

#include <math.h>
#include <stdint.h>

#include "fh_fft.h"  // FH_HD

namespace fh {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

constexpr uint64_t kTagPath = 0;
constexpr uint64_t kTagGibbs = 1;
constexpr uint64_t kTagLocal = 2;  // local link updates; pass k uses kTagLocal + 256 k
constexpr uint64_t kTagMala = 3;        // MALA proposal noise per (site, slice)
constexpr uint64_t kTagMalaAccept = 4;  // MALA acceptance uniform per chain
constexpr uint64_t kTagPerm = 5;        // reconnection swaps; pass k uses kTagPerm + 256 k

FH_HD inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

struct u64x4 {
    uint64_t x0, x1, x2, x3;
};

FH_HD inline u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                  uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = mulhi64(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
        const uint64_t hi1 = mulhi64(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return {c0, c1, c2, c3};
}

// 53-bit uniform in [0, 1).
FH_HD inline double u01_from(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// Box-Muller standard normal: u1 in (0, 1], u2 in [0, 1).
FH_HD inline double normal_from(uint64_t x0, uint64_t x1) {
    const double u1 = (double)((x0 >> 11) + 1) * 0x1.0p-53;
    const double u2 = (double)(x1 >> 11) * 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

}  // namespace fh
