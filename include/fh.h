/*
 * fh.h — C ABI of the MI355X (gfx950) FFBS worldline-sweep library.
 *
 * The library samples the joint measure of fermion worldlines and Hubbard-Stratonovich (HS)
 * fields of the determinant-free auxiliary-variable MCMC of Kong, Feng, Xie and Wu
 * ("FFT-Accelerated Auxiliary Variable MCMC for Fermionic Lattice Models", eq. joint). The
 * worldlines close on themselves unless a permutation is set (fh_set_permutation: reconnections at
 * tau = beta with sign, Sec. 3.5.6). One sweep redraws every worldline block by forward
 * filtering / backward sampling (Sec. 3.5.2) and then every field value from its exact
 * conditional (Sec. 3.5.4 / 3.5.5).
 *
 * Conventions used by every entry point
 *  - Lattice: L x L periodic square lattice, N = L*L sites, site index i = x + L*y.
 *  - Worldlines are held in the site basis: paths[l][p] is the site of particle p on imaginary
 *    time slice l (0 <= l < L_tau); particles 0..n_up-1 are spin up, n_up..n_up+n_dn-1 spin down.
 *    A path weighs prod_l W_{l,spin}(r_l) G(r_{l+1} - r_l), G the real-space hopping kernel
 *    (inverse Fourier transform of exp(-dtau eps_k), eq. Tkk / Sec. 3.3), r_{L_tau} = r_0 of the
 *    worldline it reconnects to (itself unless a permutation is set).
 *  - Fields: aux[l][i], Gaussian sigma (FH_HS_GAUSS, eq. gaussHS) or Ising s = +-1.0
 *    (FH_HS_HIRSCH, eq. hirsch). Site potentials: Gaussian W_up = W_dn = exp(a*sigma),
 *    a = sqrt(|U| dtau); Ising W_up = exp(lambda*s), W_dn = exp(-lambda*s),
 *    cosh(lambda) = exp(dtau U / 2).
 *  - Batches: a plan holds n_chains independent chains, possibly of different shapes. All
 *    per-chain arrays are packed one chain after the other; fh_layout() gives the offsets.
 *      aux      : sum_c L_tau*N elements, double (FH_FP64) or float (FH_FP32, FH_FP32_MFMA3)
 *      paths    : sum_c L_tau*n_particles int32
 *      logZ     : sum_c n_particles double (per particle)
 *  - Memory: every array argument is a DEVICE pointer, owned by the caller, that must stay
 *    valid until the work queued on `stream` has finished. The plan owns only its workspace.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream). Calls enqueue work and
 *    return without synchronising, except fh_get_status and fh_get_filters' row count.
 *  - Errors: every call returns FH_OK (0) or a negative code. Argument and state errors are
 *    reported synchronously; errors found by kernels (non-finite weights, a zero total weight,
 *    a site index out of range in `paths`) are latched in a device status word that
 *    fh_get_status reads. A plan is not thread-safe; calls on one plan must be serialised.
 *  - Random numbers: Philox4x64-10 (Salmon et al., SC'11), key (seed, 0), counter
 *    (index, slice, sweep, tag); tag 0: one uniform per (particle, slice, sweep) for backward
 *    sampling, tag 1: one draw per (site, slice, sweep) for the field. Results therefore depend
 *    only on (state, sweep index, seed), not on batch composition or launch shape.
 */
#ifndef FH_H
#define FH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fh_plan_s* fh_plan;
typedef void* fh_stream; /* hipStream_t */

enum fh_status {
    FH_OK = 0,
    FH_ERR_INVALID_ARG = -1, /* bad descriptor, null pointer, size or index           */
    FH_ERR_UNSUPPORTED = -2, /* valid request the library does not implement (e.g. L) */
    FH_ERR_OOM = -3,         /* device allocation failed                               */
    FH_ERR_HIP = -4,         /* a HIP runtime call failed                              */
    FH_ERR_NONFINITE = -5,   /* device: a normaliser or weight total was NaN or Inf    */
    FH_ERR_ZERO_WEIGHT = -6, /* device: a backward-sampling weight total was zero      */
    FH_ERR_STATE = -7,       /* call order violated (e.g. backward before forward)     */
    FH_ERR_BAD_PATH = -8     /* device: a site index in `paths` was outside [0, N)     */
};

enum fh_hs_kind { FH_HS_GAUSS = 0, FH_HS_HIRSCH = 1 };

enum fh_precision {
    FH_FP64 = 0,      /* plain path: FP64 FFT convolution, FP64 filters                       */
    FH_FP32 = 1,      /* FP32 FFT convolution and filters; FP64 normaliser and CDF            */
    FH_FP32_MFMA3 = 2 /* FP32 filters, convolution as the separable real circulant on MFMA
                         with three-term split-bf16 products; FP64 normaliser and CDF;
                         32 < L < 64 zero-padded to 64 (fh_logZ_grad and fh_mala_field:
                         L <= 32)                                                             */
};
/* Range of the FP32 plans. A filter row is normalised to sum 1; FP32 holds its values to full
 * relative precision only down to ~2^-110 (bf16 splitting) or ~2^-126. Strong, clustered fields
 * push the part of a row that a block's draws need below that (block end weights of 2^-160 and
 * less occur on the way to clustered states). Both FP32 plans therefore hold W and the filter
 * rows scaled high in FP32's range, queue every block whose forward step loses nearly all its
 * mass to the weights (below 2^-196 of it), whose end weight falls below 2^-110 of the row mass
 * or whose backward draw picks a site with a filter value below that, queue every block of a
 * chain that has a queued block (in that pass and the next two), and redo the
 * queued blocks in FP64: the forward recursion on the FP64 circulant with W computed in FP64 from
 * the field (its log Z replaces the FP32 one, its rows rounded to FP32 replace the stored rows),
 * and, in fh_backward_sample and fh_sweep, the block's draws from the FP64 rows with the same
 * rule and uniforms as an FH_FP64 plan. Only chains with L <= 32, L = 48 or L = 64 have this
 * FP64 re-filter; a queued block of another lattice latches FH_ERR_NONFINITE and keeps its
 * sites. */

enum fh_flags {
    FH_FLAG_NONE = 0,
    FH_FLAG_GRAPH = 1,   /* fh_sweep replays a captured hipGraph instead of eager launches     */
    FH_FLAG_AUTOTUNE = 2, /* fh_init times every radix-2/3/4 stage order of each distinct L on
                            the device (FFT precisions) and keeps the fastest; without it the
                            default order (4s, then a 2, then 3s) is used                    */
    FH_FLAG_FFT_CONV = 8, /* FH_FP64 plans convolve every chain with the FP64 FFT. Without it
                            chains with L <= 32, 48 or 64 use the circulant C f C on the FP64
                            matrix cores (every product positive, so filter tails keep their
                            relative accuracy); other L > 32 always use the FFT                */
    FH_FLAG_FULL_ROW_DRAW = 4, /* backward draws scan every site of the filter row. Without it a
                            chain whose hopping kernel decays fast enough draws from the window
                            of sites within w <= 3 steps of the next slice's site and certifies
                            that the draw equals the full-row one (else scans the row): the
                            same draws, fewer bytes read. While the window leaves more than
                            3/20 of a backward pass's draws uncertified (clustered states), the
                            plan draws the following passes with the full-row kernels and
                            retries the window after 16 to 64 passes; the draws are the same */
    FH_FLAG_GRAD_CHECKPOINT = 16 /* the adjoint (fh_logZ_grad, fh_kinetic_energy,
                            fh_mala_field) keeps every K-th ring row, K = ceil(sqrt(L_tau)), and
                            recomputes each segment of K rows from its checkpoint during the
                            backward messages: about 2 sqrt(L_tau) rows per worldline instead
                            of L_tau, for one more forward recursion; the results are the
                            same bits. The filter workspace of the sweep (L_tau rows per
                            worldline) is then allocated only by the first fh_forward_filter
                            or fh_sweep, and fh_get_filters returns FH_ERR_STATE after the
                            adjoint. Needs the matrix-core adjoint: FH_FP32_MFMA3, or FH_FP64
                            without FH_FLAG_FFT_CONV, every chain with L <= 32 (else fh_init
                            returns FH_ERR_UNSUPPORTED)                                       */
};

/* One chain. block_len: FFBS block length B (0 = L_tau, one block closing the ring);
 * blocks of a sweep s start at o_s + j*B (mod L_tau), o_s = (s*floor(B/2)) mod L_tau,
 * the last one shorter when B does not divide L_tau; endpoints stay fixed within a sweep.
 * Requirements: L in {2..64} with L = 2^a 3^b, L_tau >= 2,
 * n_up, n_dn >= 0 with n_up + n_dn >= 1, block_len = 0 or 2 <= block_len <= L_tau,
 * t > 0, dtau > 0, U finite (U >= 0 for FH_HS_HIRSCH), all finite. */
typedef struct {
    int32_t L, L_tau, n_up, n_dn, hs_kind, block_len;
    double t, U, dtau;
    uint64_t seed;
} fh_chain_desc;

/* Element offsets and counts of one chain inside the packed batch arrays. */
typedef struct {
    int64_t aux_offset, aux_count;           /* aux: L_tau*N elements            */
    int64_t path_offset, path_count;         /* paths: L_tau*n_particles int32   */
    int64_t particle_offset;                 /* per-particle arrays (logZ)       */
    int32_t L, N, L_tau, n_particles;
} fh_chain_layout;

/* Creates a plan for n_chains chains: validates every descriptor, builds the hopping tables
 * (exp(-dtau eps_k) of Sec. 3.3 and its real-space kernel), picks the FFT radix plan per L
 * (timed on the device with FH_FLAG_AUTOTUNE) and allocates the workspace (filters of every particle: L_tau*N values each in the plan's
 * precision). Synchronous. *out is NULL on failure. */
int fh_init(fh_plan* out, const fh_chain_desc* descs, int32_t n_chains, int32_t precision,
            uint32_t flags);
int fh_destroy(fh_plan plan);

/* The FFT radix plan of chain `chain` (both dimensions): n_stages stages with radices
 * radices[0..n_stages) in {2, 3, 4}, product L, applied in that order by every Stockham FFT of
 * the chain (forward filter and adjoint of the FH_FP64 / FH_FP32 paths; unused on
 * FH_FP32_MFMA3). radices: host array of at least 6 int32. Stage order is the only choice the
 * autotuner makes; the transform is the same up to rounding for every order. */
int fh_get_radix_plan(fh_plan plan, int32_t chain, int32_t* radices, int32_t* n_stages);

/* Layout of chain `chain` in the packed arrays; totals over the batch via fh_sizes. */
int fh_layout(fh_plan plan, int32_t chain, fh_chain_layout* out);
int fh_sizes(fh_plan plan, int64_t* aux_elems, int64_t* path_elems, int64_t* particles);

/* Forward filtering (Sec. 3.5.2, eq. ffbsFwd, site basis) of every block of every particle
 * for sweep `sweep`, given the field `aux` and the current worldlines `paths` (read for the
 * block endpoints only): f_0 = W(a) delta_a, f_j = W . (G * f_{j-1}), each f_j rescaled by its
 * sum with the logarithms accumulated in FP64; the normalised filters stay in the plan for
 * fh_backward_sample. logZ (nullable): per particle, the sum over its blocks of
 * log Z_block = log [(G * f_{n-1})(end site)]. */
int fh_forward_filter(fh_plan plan, const void* aux, const int32_t* paths, uint64_t sweep,
                      double* logZ, fh_stream stream);

/* Backward sampling (Sec. 3.5.2, the exact conditional P(r_j | r_{j+1}) ∝ f_j(r) G(r_{j+1}-r))
 * of every block interior, from the filters of the last fh_forward_filter, which must have been
 * called with the same `sweep` and the same `paths` contents (FH_ERR_STATE otherwise).
 * Inverse CDF in site order with an FP64 running sum; the draw is the smallest site whose
 * running sum exceeds u * total. `paths` is updated in place (block endpoints are kept).
 * FP32 plans re-filter out-of-range blocks (see the range note above) from the `aux` passed to
 * that fh_forward_filter, which must therefore still hold the same field. */
int fh_backward_sample(fh_plan plan, int32_t* paths, uint64_t sweep, fh_stream stream);

/* Exact Gibbs draw of the whole field given the worldlines (Sec. 3.5.4: Ising,
 * P(s=+1) = (1 + tanh(lambda m))/2, m = n_up - n_dn; Sec. 3.5.5, eq. gaussCond: Gaussian,
 * sigma ~ N(a (n - 1/2), 1), n = n_up + n_dn), counts taken from `paths`. `aux` is overwritten. */
int fh_gibbs_aux(fh_plan plan, const int32_t* paths, void* aux, uint64_t sweep,
                 fh_stream stream);

/* Local link updates (Sec. 3.5.1, eq. Rlocal, site basis): n_passes Metropolis passes; a pass
 * is a checkerboard in tau: it visits the odd interior slices l = 1, 3, ... <= L_tau-2 of every
 * worldline, then the even interior slices 2, 4, ... <= L_tau-2, then slice 0 of every
 * worldline, then slice L_tau-1 of every worldline (the end slices neighbour the worldlines the
 * reconnection at tau = beta links to). The visits of one phase are independent of each other.
 * Each visit proposes moving the worldline's site r on slice l to a nearest neighbour r' (+x,
 * -x, +y or -y, equally likely, periodic) with its sites on slices l-1 and l+1 fixed (as left by
 * the earlier phases), and takes it iff u < R,
 * R = W_l(r') G(r' - r_{l-1}) G(r_{l+1} - r') / [W_l(r) G(r - r_{l-1}) G(r_{l+1} - r)], in FP64.
 * Random numbers: Philox counter (particle, slice, sweep, 2 + 256*pass); the top two bits of
 * word 1 pick the direction, word 0 gives u. aux is read, paths updated in place. The filters of
 * the last fh_forward_filter are invalidated (fh_backward_sample then returns FH_ERR_STATE).
 * n_passes = 0 does nothing; negative is FH_ERR_INVALID_ARG. */
int fh_local_update(fh_plan plan, const void* aux, int32_t* paths, uint64_t sweep,
                    int32_t n_passes, fh_stream stream);

/* Reconnections of the worldlines at tau = beta (eq. joint's sum over permutations; Sec. 3.5.6).
 * The plan holds one permutation per spin of every chain: slice L_tau of worldline p is slice 0
 * of worldline perm[p] (chain-local indices, up worldlines mapped onto up worldlines and down onto
 * down), and a sign sgn(P_up) sgn(P_dn) per chain by which observables are reweighted (the
 * sampled measure is |pi|). fh_init starts from the identity, sign +1. FFBS blocks that run past
 * slice L_tau - 1 continue on the reconnected worldline (their end site is read from it and their
 * interior slices from L_tau on are written to it); local updates link slice L_tau-1 of p to
 * slice 0 of perm[p]. fh_logZ_grad and fh_mala_field close the ring of worldline p on the anchor
 * site of perm[p]: Z_p sums the paths from p's anchor site to that of perm[p] over L_tau slices. */

/* Sets the permutation from a host array [particles] (packed like logZ: chain c's entries at its
 * particle_offset) and recomputes the signs. FH_ERR_INVALID_ARG unless every chain's entries are
 * a permutation of its worldlines that maps each spin onto itself. Synchronous. */
int fh_set_permutation(fh_plan plan, const int32_t* perm);

/* Copies the permutation (host array [particles], nullable) and the per-chain signs (host array
 * [n_chains], nullable) out of the plan. Synchronous. */
int fh_get_permutation(fh_plan plan, int32_t* perm, int32_t* sign);

/* n_passes passes of pair swaps of the reconnections (Sec. 3.5.6): pass k pairs the worldlines of
 * each spin as (p0 + o + 2i, p0 + o + 2i + 1), o = k mod 2 (p0 the spin's first worldline); a pair
 * (p, q) trades perm[p] and perm[q] iff u < R, R the ratio of the two boundary hops after and
 * before, G(r^{P(q)}_0 - r^p_{L-1}) G(r^{P(p)}_0 - r^q_{L-1}) / [G(r^{P(p)}_0 - r^p_{L-1})
 * G(r^{P(q)}_0 - r^q_{L-1})] in FP64, u from the Philox counter (p, 0, sweep, 5 + 256 k). Every
 * accepted swap flips the chain's sign. paths is read only. */
int fh_permutation_update(fh_plan plan, const int32_t* paths, uint64_t sweep, int32_t n_passes,
                          fh_stream stream);

/* Equal-time observables of the worldlines `paths` (Sec. 4), per chain, averaged over the
 * slices: with S^z_j = (n_{j,up} - n_{j,dn}) / 2 (worldline counts per site),
 *   S(k) = (1/N) |sum_j e^{i k.r_j} S^z_j|^2,   k = 2 pi (k_x, k_y) / L indexed k_x + L k_y,
 *   C(r) = (1/N) sum_j S^z_{j+r} S^z_j,         r indexed x + L y,
 *   D = mean over sites of n_up n_dn,  S2 = (3/4) mean over sites of (n_up - n_dn)^2.
 * S(k) and C(r) come from one FP64 2D FFT of S^z per slice and one inverse FFT of |F|^2. Outputs
 * are device arrays, each nullable: Sk and Cr packed by chain (chain c's N_c values after those
 * of chains 0..c-1), D and S2 [n_chains]. The first call allocates the plan's per-slice rows
 * (2 * aux elements + 2 * slices doubles). */
int fh_measure(fh_plan plan, const int32_t* paths, double* Sk, double* Cr, double* D,
               double* S2, fh_stream stream);

/* fh_measure for callers that cannot allocate device memory (code under stream capture, serving
 * loops, harnesses that forbid it): the same kernels, outputs and arguments, with the per-slice
 * rows in a static device array of 2^22 doubles (32 MiB) that every GPU the library runs on holds
 * until the process ends, instead of a buffer the plan allocates on first use. The call itself
 * calls no allocator. Returns FH_ERR_UNSUPPORTED when the plan needs more than the array holds
 * (2 * aux elements + 2 * slices of all chains > 2^22, e.g. more than 12 chains of 32 x 32 with
 * L_tau = 160) and FH_ERR_HIP when the array's address could not be taken at fh_init. All calls
 * on one GPU share its array: calls that overlap in time on one GPU (any plans, any streams)
 * race and must be serialised by the caller. */
int fh_measure_noalloc(fh_plan plan, const int32_t* paths, double* Sk, double* Cr, double* D,
                       double* S2, fh_stream stream);

/* n_sweeps full sweeps, sweep indices first_sweep .. first_sweep+n_sweeps-1: forward filter,
 * backward sample, Gibbs field draw, in place on aux and paths. With FH_FLAG_GRAPH the sweep
 * is captured once per (aux, paths) pair and replayed. */
int fh_sweep(fh_plan plan, void* aux, int32_t* paths, uint64_t first_sweep, int32_t n_sweeps,
             fh_stream stream);

/* log Z_path and its gradient. log Z_path = sum_p log Z_p, Z_p the weight of all closed paths
 * of particle p through its current site at slice anchor_slice (one block of length L_tau),
 * i.e. log p(anchor sites | field) + const; the HS prior is excluded. Hand-written adjoint:
 * backward messages beta_j = G * (W_{j+1} . beta_{j+1}), d log Z / d log W_j(r) =
 * f_j(r) beta_j(r) / Z, d/dt through d exp(-dtau eps_k)/dt in Fourier space.
 * logZ: per chain [n_chains] (nullable); grad_aux: packed like aux, overwritten, in the
 * plan's precision, d log Z_path / d aux(l, r) (nullable); grad_t: [n_chains] (nullable).
 * Every adjoint writes one partial field gradient per group of worldlines and adds a chain's
 * groups in a fixed order, so repeated calls on the same inputs return the same bits. */
int fh_logZ_grad(fh_plan plan, const void* aux, const int32_t* paths, int32_t anchor_slice,
                 double* logZ, void* grad_aux, double* grad_t, fh_stream stream);

/* Rao-Blackwellised kinetic energy per chain (the expectation of the hopping term of the Hubbard
 * Hamiltonian, eq. hubbard, with the worldlines' paths summed out given their sites at
 * anchor_slice): energy[c] = -(t_c / beta_c) d log Z_path / d t_c, beta_c = L_tau dtau, Z_path
 * as in fh_logZ_grad; t enters each kinetic step through exp(-dtau eps_k) of the symmetric
 * Trotter split (Sec. on the path integral). The paper gives no estimator of its own; this is
 * the one its path weights define. energy: device double [n_chains], overwritten. Same
 * argument rules, errors and filter side effects as fh_logZ_grad; fixed-order reductions. */
int fh_kinetic_energy(fh_plan plan, const void* aux, const int32_t* paths, int32_t anchor_slice,
                      double* energy, fh_stream stream);

/* One gradient-informed move of the Gaussian field of every chain: a Metropolis-adjusted Langevin
 * step (Roberts and Tweedie, 1996) on the field's law given the worldlines' sites at
 * anchor_slice with their paths summed out,
 *   pi(sigma) ∝ prod_{r,l} exp(-sigma^2/2 - a sigma/2) * Z_path(sigma)   (eq. gaussHS prior,
 *   Z_path as in fh_logZ_grad):
 *   sigma' = sigma + h g(sigma) + eps xi,  h = eps^2/2,  g = d log pi / d sigma,
 * xi_rl ~ N(0,1) from the Philox counter (site, slice, sweep, 3) by Box-Muller; the chain's whole
 * field moves to sigma' iff u < min(1, alpha), alpha the Metropolis-Hastings ratio with the
 * Langevin proposal densities, u from counter (0, 0, sweep, 4). Two log Z_path-and-gradient
 * evaluations per call. aux (plan precision, device) is updated in place; accepted (device
 * int32 [n_chains], nullable) receives 1 or 0, and -1 for Ising-field chains, which stay
 * unchanged. eps > 0 and finite. The first call allocates three field-sized work arrays. The
 * step is an exact Metropolis-Hastings step on an FH_FP64 plan; on the FP32 plans log Z_path
 * carries the FP32 filter error, which makes the acceptance approximate. */
int fh_mala_field(fh_plan plan, void* aux, const int32_t* paths, int32_t anchor_slice,
                  double eps, uint64_t sweep, int32_t* accepted, fh_stream stream);

/* Replaces the hopping amplitude of every chain (t: host array [n_chains], each > 0) and
 * rebuilds the kernel tables. Synchronous; invalidates stored filters. */
int fh_set_hopping(fh_plan plan, const double* t);

/* Synchronises the device and returns the first device-side error latched since the last
 * call (FH_OK if none) and the chain it occurred in (-1 if none); clears the latch. */
int fh_get_status(fh_plan plan, int32_t* code, int32_t* first_chain);

/* Copies the normalised filter rows stored for (chain, particle) by the last forward filter
 * into dst (device, capacity elements of the plan's precision). Rows are N values each:
 * for fh_forward_filter the interior rows j = 1..n-1 of each block in block order
 * (L_tau - n_blocks rows); after fh_logZ_grad the L_tau rows j = 0..L_tau-1 of the ring.
 * *n_rows receives the row count. Synchronous. */
int fh_get_filters(fh_plan plan, int32_t chain, int32_t particle, void* dst, int64_t capacity,
                   int64_t* n_rows, fh_stream stream);

/* Static description of an error code. */
const char* fh_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* FH_H */
