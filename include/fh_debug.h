/*
 * fh_debug.h — host-only diagnostic entry points of the FFBS library.
 *
 * These run entirely on the CPU, with the same source as the device code paths they mirror,
 * so that index arithmetic can be checked without a GPU. They are not part of the sampling
 * path and allocate nothing on the device.
 */
#ifndef FH_DEBUG_H
#define FH_DEBUG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 2D FFT of an L x L complex tile (interleaved re, im; element (x, y) at index x + L*y), run on
 * the host with the GPU kernels' Stockham stage code and radix plan. inverse = 0: forward
 * (exp(-2 pi i k.n / L)); inverse = 1: conjugate twiddles, unscaled. data is overwritten.
 * Returns FH_OK or FH_ERR_UNSUPPORTED (L not 2^a 3^b in [2, 64]). */
int fh_debug_fft2d_host(double* data, int32_t L, int32_t inverse);

/* Real-space hopping kernel table g(d), d = 0..L-1, as built by fh_init (modified Bessel
 * series). out: host array of L doubles. */
int fh_debug_kernel_table(int32_t L, double t, double dtau, double* out);

/* Philox4x64-10 block for counter (c0..c3) and key (k0, k1), computed on the host with the
 * library's generator. out: host array of 4 uint64. */
int fh_debug_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                    uint64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* FH_DEBUG_H */
