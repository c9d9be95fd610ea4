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

#include "fh.h"

#ifdef __cplusplus
extern "C" {
#endif

/* 2D FFT of an L x L complex tile (interleaved re, im; element (x, y) at index x + L*y), run on
 * the host with the GPU kernels' Stockham stage code and radix plan. inverse = 0: forward
 * (exp(-2 pi i k.n / L)); inverse = 1: conjugate twiddles, unscaled. data is overwritten.
 * Returns FH_OK or FH_ERR_UNSUPPORTED (L not 2^a 3^b in [2, 64]). */
int fh_debug_fft2d_host(double* data, int32_t L, int32_t inverse);

/* Same as fh_debug_fft2d_host with an explicit stage order: n_stages radices from {2, 3, 4}
 * whose product is L (any order the autotuner may pick). FH_ERR_INVALID_ARG otherwise. */
int fh_debug_fft2d_host_plan(double* data, int32_t L, const int32_t* radices, int32_t n_stages,
                             int32_t inverse);

/* The autotuner's candidates for L: every ordered sequence of radices from {2, 3, 4} with
 * product L and at most 6 stages, each once. out: host array of cap * 7 int32, entry k =
 * (n_stages, radix_0, ..., radix_5) with unused radices 0. Returns the number of candidates
 * (0 when L is not 2^a 3^b in [2, 64]); only the first cap are written. */
int fh_debug_radix_orders(int32_t L, int32_t* out, int32_t cap);

/* Real-space hopping kernel table g(d), d = 0..L-1, as built by fh_init (modified Bessel
 * series). out: host array of L doubles. */
int fh_debug_kernel_table(int32_t L, double t, double dtau, double* out);

/* Philox4x64-10 block for counter (c0..c3) and key (k0, k1), computed on the host with the
 * library's generator. out: host array of 4 uint64. */
int fh_debug_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                    uint64_t* out);

/* Window selection for backward draws from a kernel table g[0..L): writes the half-width w
 * (1..3) and g_out, the bound on G(s - r) = g(dx) g(dy) over sites r outside the window of s.
 * Returns 1 when w qualifies (window covers the lattice, or g_out <= 2^-20 max G), 0 when not
 * (w = 3 with its true bound), FH_ERR_INVALID_ARG on bad input. */
int fh_debug_window_select(const double* g, int32_t L, int32_t* w, double* g_out);

/* One backward draw on the host with the windowed rule of the backward kernel: f is a filter row
 * [L*L] (site x + L*y), s_site the next slice's site, u in [0, 1). Weights max(f, 0) g(dy) g(dx).
 * *certified = 1 when the window's draw carried its certificate against the outside bound
 * g_out, 2 when the wider second window (half-width 7, its bound computed from g) certified it,
 * 0 when the draw was taken over the full row (first cumulative weight above u times the total,
 * else the last positive weight). Returns FH_OK, FH_ERR_ZERO_WEIGHT, FH_ERR_NONFINITE or
 * FH_ERR_INVALID_ARG. */
int fh_debug_window_draw(int32_t L, int32_t w, const double* g, double g_out, const double* f,
                         int32_t s_site, double u, int32_t* site, int32_t* certified);

/* Device-plan test hooks (they synchronise the device):
 *   fh_debug_inflate_window_bound multiplies every chain's outside bound by factor >= 1 (an
 *   infinite factor sends every windowed draw through the full-row scan; a larger bound only
 *   makes the certificate stricter, so draws stay exact);
 *   fh_debug_backward_kernels reports how many backward tasks belong to chains that may use the
 *   windowed kernel (n_windowed) and how many to chains that always use the full-row kernels
 *   (n_full_row);
 *   fh_debug_backward_adapt switches the plan's choice between the windowed and the full-row
 *   kernels on (enable = 1, the default of a new plan) or off (0: windowed chains always use the
 *   window). After a backward pass whose first windows left more than 3/20 of the windowed
 *   chains' draws uncertified, the next backward passes (16, doubling to 64 while retries fail)
 *   use the full-row kernels; the draws are the same either way. full_row_passes_left (nullable,
 *   caller-owned, one int32) receives how many coming backward passes use the full-row kernels
 *   (0: the window), read before the switch; changing the setting puts the plan back on the
 *   window. */
int fh_debug_inflate_window_bound(fh_plan plan, double factor);
int fh_debug_backward_kernels(fh_plan plan, int32_t* n_windowed, int32_t* n_full_row);
int fh_debug_backward_adapt(fh_plan plan, int32_t enable, int32_t* full_row_passes_left);

/* FP32 plans queue the blocks whose filters leave FP32's range (see the range note of fh.h),
 * and every block of a chain that had such a block in this or one of the four preceding forward
 * passes, for an FP64 re-filter and redraw (the FP32 forward kernels skip the chains held so). fh_debug_rescue synchronises the device and reports
 * the queue of the last forward pass (with what its backward pass added): last_count
 * (nullable) receives its length, whole_chains (nullable) the chains queued whole, total
 * (nullable) the blocks redrawn by every backward pass since the previous call (then reset to
 * 0), and list (caller-owned host memory, cap triples, may be null when cap = 0) the first
 * min(cap, last_count) queued blocks as (chain, particle, block). FP64 plans report 0. */
int fh_debug_rescue(fh_plan plan, int32_t* last_count, int32_t* whole_chains, int64_t* total,
                    int32_t* list, int32_t cap);
/* Overwrites every value of stored filter row `row` (numbered as fh_get_filters returns them) of
 * (chain, particle) with `value`, in the plan's precision; the host's way to force a row whose
 * backward weights are all zero. Needs stored filters (FH_ERR_STATE otherwise). Synchronous. */
int fh_debug_fill_filter_row(fh_plan plan, int32_t chain, int32_t particle, int32_t row,
                             double value);
/* Shared forward filters (FP32 matrix-core plans, 32 x 32 chains): the worldlines of one
 * (chain, spin, block) with the same start site share the stored rows of the lowest of them,
 * their representative. Synchronises the device and copies the representative map of the last
 * forward pass, one chain-local particle index per (chain, particle, block) at
 * blk_off + p * n_blocks + b (chain after chain, fh_layout's particle order), to rep
 * (caller-owned host memory, min(cap, *n) entries). *n receives the map's length: 0 when no
 * chain of the plan shares filters (then every worldline reads its own rows). */
int fh_debug_representatives(fh_plan plan, int32_t* rep, int64_t cap, int64_t* n);
/* enable = 0: every worldline runs its own forward recursion (the representative map is the
 * identity), the reference for tests that the shared filters change no result; 1 (the
 * default): shared. Synchronous; drops the captured sweep and invalidates stored filters. */
int fh_debug_share_filters(fh_plan plan, int32_t enable);
/* Synchronises the device and writes to holds (caller-owned host memory, [n_chains]) the forward
 * passes each chain stays on the FP64 re-filter: a chain with L <= 32 and holds[c] > 0 is
 * skipped by the next forward pass's FP32 kernels and re-filtered whole. FP64 plans write 0. */
int fh_debug_rescue_holds(fh_plan plan, int32_t* holds);

/* FP32 plans: why the kernels queued blocks for the FP64 re-filter, counted since fh_init (a
 * block met by several floors, or in several passes, counts each time): counts[0] a forward
 * step's W-weighted mass below the step floor (or not finite), counts[1] an end weight below
 * the range floor, counts[2] a backward draw at a site whose filter value is below the range
 * floor (or with no positive weight), counts[3] the FP32 FFT forward (either floor). counts
 * holds 4 int32 written by the call (caller-owned host memory; zeros on FP64 plans). */
int fh_debug_rescue_causes(fh_plan plan, int32_t* counts);

/* Per-sweep timing for the benchmark: with enable = 1, every sweep of fh_sweep records HIP events
 * of the plan around its forward-filter kernels, its backward-sampling kernels and the FP64
 * re-filter of out-of-range blocks (FP32 plans); the sweeps are then launched eagerly (the same
 * kernels on the same streams) instead of from the captured graph, whose event nodes cannot be
 * timed. fh_debug_sweep_times waits for the last sweep and writes four durations in
 * milliseconds to ms[0..3] (caller-owned host memory): the forward kernels, the backward
 * kernels, the FP64 re-filter on the caller's stream (including the wait for its phase A), and
 * phase A, the re-filter of the chains held on FP64 on the plan's side stream, which runs beside
 * the first two (0 on FP64 plans). */
int fh_debug_sweep_timing(fh_plan plan, int32_t enable);
int fh_debug_sweep_times(fh_plan plan, float* ms);

/* Forward work items of an FH_FP32_MFMA3 plan, by kernel: counts[0] worldline pairs of L = 32
 * chains, counts[1] single padded worldlines (16 < L < 32), counts[2] packed tasks of 2 x 2
 * worldlines per tile (8 < L <= 16), counts[3] packed tasks of 4 x 4 (L <= 8), counts[4] single
 * worldlines of L = 64 chains on four 32 x 32 sub-tiles, counts[5] single worldlines of
 * 32 < L < 64 chains on the same sub-tiles, zero-padded. counts holds 6 int32 written by the
 * call (caller-owned host memory). */
int fh_debug_forward_kernels(fh_plan plan, int32_t* counts);

#ifdef __cplusplus
}
#endif

#endif /* FH_DEBUG_H */
