// Forward filter on the matrix cores (FH_FP32_MFMA3): the kinetic step as the separable real
// circulant H = C F C with C[i][j] = g(i - j mod L), computed with v_mfma_f32_32x32x16_bf16
// and three-term split-bf16 operands.
//
// Why a circulant and not an FFT here: the kernel G(d) = g(d_x) g(d_y) is positive, so the
// direct products carry relative (not max-relative) rounding error and FP32 filters stay far
// inside 1e-5 over hundreds of slices, where FP32 FFT round-off drifts coherently past it.
//
// Layout. One wavefront owns one worldline's L x L filter zero-padded to a 32 x 32 tile, in
// the MFMA accumulator layout: lane l, register v holds X[rho(l, v)][l % 32] with
// rho = 8 (v / 4) + 4 (l / 32) + v % 4. Handing those registers straight back as the A operand
// (chunk q takes registers 8q .. 8q+7) makes the instruction see A[m][kappa] = X[R(kappa)][m]
// with R(16q + 8h + e) = 16q + 8 (e / 4) + 4h + e % 4, so with B[kappa][n] = C[R(kappa)][n]
// it computes X^T C. Two such products give (F^T C)^T C = C F C: no transpose, no LDS.
//
// Precision. F (each step) and C (once, on the host) are split into bf16 terms
// x = x_h + x_m + x_l (8 bits each, exact to ~2^-27); the six products of combined order up to
// 2^-18 (hh, hm, hl, mh, mm, lh) are accumulated in FP32. Fewer terms leave either a coherent
// bias of the kernel's mass (log Z drifts ~1e-4 over 160 slices) or a filter drift ~4e-5.
// The per-step normaliser is a DPP wavefront sum in FP32; log Z is accumulated in FP64.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "fh_dmfma.h"
#include "fh_internal.h"

namespace fh {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
static_assert(kWaves == kGroup, "one adjoint worldline (and segment) per wavefront");

__device__ inline int tile_row(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

__device__ inline void set_status(int32_t* st, int code, int chain) {
    if (atomicCAS(&st[0], 0, code) == 0) atomicExch(&st[1], chain);
}

struct Split3 {
    bf16x8 h[2], m[2], l[2];
};

typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

// (a, b) -> two bf16 (round to nearest even) packed as one dword, a in the low half.
__device__ inline uint32_t pk_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// The bf16 pairs (-1, 0) and (0, -1), for v_dot2c_f32_bf16: dot2((h_a, h_b), (-1, 0), a) is
// a - h_a, exact (the rounding error of a bf16 rounding is an FP32 number, subnormals
// included). They reach the kernels as arguments: written as a literal, the pair is folded into
// a 32-bit inline constant whose halves do not match the pair.
struct NegPairs {
    uint32_t lo, hi;
};
constexpr NegPairs kNegPairs = {0x0000BF80u, 0xBF800000u};

__device__ inline float resid_lo(uint32_t p, float a, const NegPairs& n) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, p), __builtin_bit_cast(bf16x2, n.lo), a, false);
}
__device__ inline float resid_hi(uint32_t p, float b, const NegPairs& n) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, p), __builtin_bit_cast(bf16x2, n.hi), b, false);
}

// Registers 8q .. 8q+7 of x as x = h + m + l, each term rounded to bf16 (nearest even). Works
// on pairs: one packed convert per term and one exact residual per element.
__device__ inline void split3_chunk(const f32x16& x, int q, bf16x8& h, bf16x8& m, bf16x8& l,
                                    const NegPairs& n) {
    u32x4 uh, um, ul;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float a = x[8 * q + 2 * e], b = x[8 * q + 2 * e + 1];
        const uint32_t ph = pk_bf16(a, b);
        const float ra = resid_lo(ph, a, n), rb = resid_hi(ph, b, n);
        const uint32_t pm = pk_bf16(ra, rb);
        const float sa = resid_lo(pm, ra, n), sb = resid_hi(pm, rb, n);
        uh[e] = ph;
        um[e] = pm;
        ul[e] = pk_bf16(sa, sb);
    }
    h = __builtin_bit_cast(bf16x8, uh);
    m = __builtin_bit_cast(bf16x8, um);
    l = __builtin_bit_cast(bf16x8, ul);
}

__device__ inline f32x16 mfma(const bf16x8& a, const bf16x8& b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// X (accumulator layout) -> X^T C: six split products per K chunk, smaller terms first.
__device__ inline f32x16 circ_step(const f32x16& x, const Split3& C, const NegPairs& n) {
    f32x16 acc = {};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        bf16x8 h, m, l;
        split3_chunk(x, q, h, m, l, n);
        acc = mfma(l, C.h[q], acc);
        acc = mfma(m, C.m[q], acc);
        acc = mfma(m, C.h[q], acc);
        acc = mfma(h, C.l[q], acc);
        acc = mfma(h, C.m[q], acc);
        acc = mfma(h, C.h[q], acc);
    }
    return acc;
}

// Sum over the wavefront: DPP within rows of 16 lanes, then the four row sums via readlane.
template <int CTRL>
__device__ inline float dpp_add(float v) {
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                   0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ inline float wave_sum_f32(float v) {
    v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141>(v);  // row_half_mirror
    v = dpp_add<0x140>(v);  // row_mirror
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Sum over a block's steps j = 1 .. len - 1 of the W shift of slice start + j less the rows'
// scale: the shifts' part of log Z, wavefront-uniform. Taken once after the recursion, lanes in
// parallel; a load of the shift inside the recursion stalls every step on it.
__device__ inline double block_shift_sum(const double* __restrict__ shift, int start, int len,
                                         int L_tau, double lsc, int lane) {
    double m = 0.0;
    for (int j = 1 + lane; j < len; j += 64) m += shift[(start + j) % L_tau];
    return wave_sum_f64(m) - (double)(len - 1) * lsc;
}

// One wavefront per (chain, worldline, block): the forward recursion of one block
//   f~_0 = delta_a; h_j = W~_{start+j} . (C f~_{j-1} C); c_j = sum h_j; f~_j = h_j / c_j
//   log Z = coef aux_start(a) + sum_j (log c_j + m_{start+j}) + log (C f~_{len-1} C)(e)
// storing f~_j (j >= 1) as FP32 rows of N values, like the FFT path. LFIX = 32 compiles the
// common full-tile case with constant offsets; LFIX = 0 handles any L <= 32 by zero padding.
template <int LFIX>
__device__ __forceinline__ void forward_mfma_body(
    int task, const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const uint16_t* __restrict__ cmat, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg, double* __restrict__ blk_la,
    float* __restrict__ endrow, const DrawTask* __restrict__ ctasks,
    const int32_t* __restrict__ ccount) {
    const int lane = threadIdx.x & 63;
    // with the dense list of representatives (k_dedup), wavefront i takes its entry i
    if (task >= (ccount ? *ccount : n_tasks)) return;  // whole wavefront; no barriers here
    const DrawTask t = ccount ? ctasks[task] : tasks[task];
    if (rescue_held(rsc, t.chain)) return;  // re-filtered whole in FP64 this pass
    const ChainInfo& c = chains[t.chain];
    // shared forward filters: only representatives run the recursion
    if (c.dedup && row_owner(rsc, c, t.p, t.block) != t.p) return;
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const int L = LFIX ? LFIX : c.L, N = LFIX ? LFIX * LFIX : c.N, L_tau = c.L_tau;
    // a chain with few representatives keeps its rows in the cache for the members that read
    // them next (as in k_forward_mfma2)
    const int n_rep = c.dedup ? rsc.words[kRescueChain + 3 * rsc.n_chains + t.chain] : 0;
    const bool cached = n_rep > 0 && (int64_t)n_rep * (c.B - 1) * N * 4 <= kCachedRowBytes;
    const int spin = t.p >= c.n_up ? 1 : 0;
    const float* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const double coef = spin ? c.coef_dn : c.coef_up;
    const int32_t* pc = paths + c.path_off;
    int a = pc[(int64_t)start * c.np + t.p];
    // a block that runs past slice L_tau - 1 ends on the worldline its owner reconnects to
    const int qe = start + len >= L_tau ? perm[c.part_off + t.p] : t.p;
    int e = pc[(int64_t)((start + len) % L_tau) * c.np + qe];
    if (a < 0 || a >= N || e < 0 || e >= N) {
        if (lane == 0) set_status(status, FH_ERR_BAD_PATH, t.chain);
        a = (a < 0 || a >= N) ? 0 : a;
        e = (e < 0 || e >= N) ? 0 : e;
    }
    // circulant operand, three bf16 terms, two K chunks: 16 bytes per (term, chunk, lane)
    Split3 C;
    {
        const uint4* cm = (const uint4*)(cmat + (size_t)t.chain * 3 * 2 * 64 * 8);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            C.h[q] = __builtin_bit_cast(bf16x8, cm[(0 * 2 + q) * 64 + lane]);
            C.m[q] = __builtin_bit_cast(bf16x8, cm[(1 * 2 + q) * 64 + lane]);
            C.l[q] = __builtin_bit_cast(bf16x8, cm[(2 * 2 + q) * 64 + lane]);
        }
    }
    const int x = lane & 31;
    const bool xin = LFIX ? true : x < L;
    // element (tile_row(lane, v), x) sits at lane_off + vrow(v) * L of a row
    const int lane_off = 4 * (lane >> 5) * L + x;
    auto vrow = [](int v) { return 8 * (v >> 2) + (v & 3); };
    auto inside = [&](int v) { return LFIX ? true : (xin && 4 * (lane >> 5) + vrow(v) < L); };
    auto load_w = [&](int l, float (&dst)[16]) {
        const float* Wl = Wsp + (int64_t)l * N;
        // a padded position reads site 0 (in bounds) and multiplies an exact zero of C f C
#pragma unroll
        for (int v = 0; v < 16; ++v) dst[v] = Wl[inside(v) ? lane_off + vrow(v) * L : 0];
    };
    const int ax = a % L, ay = a / L;
    // rows hold f~ 2^row_exp (the FP32 range scaling), from f_0 = 2^row_exp delta_a on
    const float sc = ldexpf(1.0f, c.row_exp);
    const double lsc = c.row_exp * 0.69314718055994530942;
    const float step_floor = c.step_floor;  // held in a register across the recursion
    f32x16 F;
#pragma unroll
    for (int v = 0; v < 16; ++v) F[v] = (x == ax && tile_row(lane, v) == ay) ? sc : 0.0f;
    double la = coef * (double)aux[c.aux_off + (int64_t)start * N + a] - lsc;
    double prod = 1.0;
    float* rows = filt + c.filt_off + ((int64_t)t.p * L_tau + (int64_t)t.block * (c.B - 1)) * N;
    // W of the next slice is loaded right after the stores of this one, so that its wait (one
    // step of matrix work later) finds the stores, which may be skipped for padded lanes and so
    // are not counted ahead of time, long retired
    // two W buffers that swap roles every step (one buffer would make the loop's back edge copy
    // the loaded slice into it, waiting for the load)
    float wa[16], wb[16];
    load_w((start + 1) % L_tau, wa);
    bool low = false;  // the block left FP32's range: queued for the FP64 re-filter
    auto step = [&](int j, const float (&wn)[16], float (&wf)[16]) {
        const int l = (start + j) % L_tau;
        const f32x16 X = circ_step(F, C, neg);
        const f32x16 H = circ_step(X, C, neg);
        float s = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            F[v] = H[v] * wn[v];
            s += F[v];
        }
        const float tot = wave_sum_f32(s);
        low |= !(tot >= step_floor) | !isfinite(tot);
        // f~_j = h_j * inv, so the normaliser actually applied is exactly 1/inv: log Z takes
        // -log(inv), accumulated as an FP64 product folded into the log occasionally; the
        // rows carry the power of two sc on top
        const float inv = __builtin_amdgcn_rcpf(tot);
        prod *= (double)inv;
        if (!(prod > 1e-200 && prod < 1e200)) {
            la -= log(prod);
            prod = 1.0;
        }
        const float k = inv * sc;
        float* row = rows + (int64_t)(j - 1) * N + lane_off;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            F[v] *= k;
            if (inside(v)) {
                if (cached)
                    row[vrow(v) * L] = F[v];
                else
                    __builtin_nontemporal_store(F[v], row + vrow(v) * L);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        load_w((l + 1) % L_tau, wf);  // the last step fetches a slice it does not use
        __builtin_amdgcn_sched_barrier(0);
    };
    if (len > 1) {
        step(1, wa, wb);
        int j = 2;
        for (; j + 1 < len; j += 2) {
            step(j, wb, wa);
            step(j + 1, wa, wb);
        }
        if (j < len) step(j, wb, wa);
    }
    la += block_shift_sum(shift, start, len, L_tau, lsc, lane);
    // end weight (C f~ C)(e)
    const f32x16 X = circ_step(F, C, neg);
    const f32x16 H = circ_step(X, C, neg);
    const int ex = e % L, ey = e / L;
    const int ve = (ey >> 3) * 4 + (ey & 3);
    const int le = ex + 32 * ((ey >> 2) & 1);
    float hv = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v)
        if (v == ve) hv = H[v];
    hv = __shfl(hv, le, 64);
    la -= log(prod);
    if (lane == 0) {
        if (low || !(hv >= kRangeFloor))
            rescue_push(rsc, c, t.chain, t.p, t.block, low ? kCauseStep : kCauseEnd);
        blk_logz[c.blk_off + (int64_t)t.p * c.nb + t.block] = la + log((double)hv);
    }
    if (c.dedup) {  // what the worldlines sharing these rows need: log Z so far, the end tile
        if (lane == 0) blk_la[c.blk_off + (int64_t)t.p * c.nb + t.block] = la;
        float* end = endrow + c.end_off + ((int64_t)t.p * c.nb + t.block) * N + lane_off;
#pragma unroll
        for (int v = 0; v < 16; ++v)
            if (inside(v)) end[vrow(v) * L] = H[v];
    }
}

template <int LFIX>
__global__ __launch_bounds__(kThreads, LFIX ? 4 : 2) void k_forward_mfma(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const uint16_t* __restrict__ cmat, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg, double* __restrict__ blk_la,
    float* __restrict__ endrow, const DrawTask* __restrict__ ctasks,
    const int32_t* __restrict__ ccount) {
    forward_mfma_body<LFIX>(
        __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6)), chains, tasks,
        n_tasks, cmat, aux, W, wshift, aux_elems, total_slices, paths, perm, filt, blk_logz,
        sweep_ptr, status, rsc, neg, blk_la, endrow, ctasks, ccount);
}

// ---- FP64 circulant on the FP64 matrix cores (fh_dmfma.h) ----------------------------------

// One wavefront per (chain, worldline, block) of an FP64 plan with L <= 32: the forward
// recursion of one block with the FP64 circulant,
//   f~_0 = delta_a; h_j = W~_{start+j} . (C f~_{j-1} C); c_j = sum h_j; f~_j = h_j / c_j
//   log Z = coef aux_start(a) + sum_j (log c_j + m_{start+j}) + log (C f~_{len-1} C)(e),
// rows f~_j (j >= 1) stored as FP64 rows of N values, exactly where the FFT path stores them.
// Padded positions (x or y >= L) stay exact zeros: C is zero outside the lattice.
__global__ __launch_bounds__(kThreads) void k_forward_dmfma(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const double* __restrict__ cmat64, const double* __restrict__ aux, const double* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, double* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status) {
    const int lane = threadIdx.x & 63;
    const int task = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    if (task >= n_tasks) return;  // whole wavefront; no barriers in this kernel
    const DrawTask t = tasks[task];
    const ChainInfo& c = chains[t.chain];
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const int L = c.L, N = c.N, L_tau = c.L_tau;
    const int spin = t.p >= c.n_up ? 1 : 0;
    const double* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const double coef = spin ? c.coef_dn : c.coef_up;
    const int32_t* pc = paths + c.path_off;
    int a = pc[(int64_t)start * c.np + t.p];
    // a block that runs past slice L_tau - 1 ends on the worldline its owner reconnects to
    const int qe = start + len >= L_tau ? perm[c.part_off + t.p] : t.p;
    int e = pc[(int64_t)((start + len) % L_tau) * c.np + qe];
    if (a < 0 || a >= N || e < 0 || e >= N) {
        if (lane == 0) set_status(status, FH_ERR_BAD_PATH, t.chain);
        a = (a < 0 || a >= N) ? 0 : a;
        e = (e < 0 || e >= N) ? 0 : e;
    }
    double Cb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) Cb[q] = cmat64[((int64_t)t.chain * 16 + q) * 64 + lane];
    const double la = coef * aux[c.aux_off + (int64_t)start * N + a];
    double* rows = filt + c.filt_off + ((int64_t)t.p * L_tau + (int64_t)t.block * (c.B - 1)) * N;
    auto wtab = [&](int l, double (&w)[16]) {
        const double* Wl = Wsp + (int64_t)l * N;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {  // a padded position reads site 0 (in bounds), times 0
                const int x = t64_x(q, lane), y = t64_y(q, r, lane);
                w[4 * q + r] = Wl[(x < L && y < L) ? y * L + x : 0];
            }
    };
    auto put = [&](int j, int q, int r, double v) {
        rows[(int64_t)(j - 1) * N + t64_y(q, r, lane) * L + t64_x(q, lane)] = v;
    };
    bool ok = true;
    const double lz = dmfma_block_forward(Cb, L, L_tau, start, len, a, e, la, shift, wtab, put, &ok);
    if (lane == 0) {
        if (!ok) set_status(status, FH_ERR_NONFINITE, t.chain);
        blk_logz[c.blk_off + (int64_t)t.p * c.nb + t.block] = lz;
    }
}

// k_forward_dmfma for the chains with L = 16 NT, NT = 3 or 4 (48 x 48, 64 x 64): the same
// recursion on NT x NT tiles of 16 x 16 with the block-circulant operands (fh_dmfma.h). The
// filter and its product take 2 NT^2 accumulator tiles (256 registers at NT = 4), so one
// wavefront runs per SIMD.
template <int NT>
__global__ __launch_bounds__(kThreads, 1) void k_forward_dmfma_big(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const double* __restrict__ cmat64, const double* __restrict__ aux, const double* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, double* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status) {
    constexpr int L = 16 * NT, N = L * L, NQ = NT * NT;
    const int lane = threadIdx.x & 63;
    const int task = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    if (task >= n_tasks) return;  // whole wavefront; no barriers in this kernel
    const DrawTask t = tasks[task];
    const ChainInfo& c = chains[t.chain];
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const int L_tau = c.L_tau;
    const int spin = t.p >= c.n_up ? 1 : 0;
    const double* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const double coef = spin ? c.coef_dn : c.coef_up;
    const int32_t* pc = paths + c.path_off;
    int a = pc[(int64_t)start * c.np + t.p];
    const int qe = start + len >= L_tau ? perm[c.part_off + t.p] : t.p;  // reconnection
    int e = pc[(int64_t)((start + len) % L_tau) * c.np + qe];
    if (a < 0 || a >= N || e < 0 || e >= N) {
        if (lane == 0) set_status(status, FH_ERR_BAD_PATH, t.chain);
        a = (a < 0 || a >= N) ? 0 : a;
        e = (e < 0 || e >= N) ? 0 : e;
    }
    double Cb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) Cb[q] = cmat64[((int64_t)t.chain * 16 + q) * 64 + lane];
    const double la = coef * aux[c.aux_off + (int64_t)start * N + a];
    double* rows = filt + c.filt_off + ((int64_t)t.p * L_tau + (int64_t)t.block * (c.B - 1)) * N;
    auto wtab = [&](int l, double (&w)[4 * NQ]) {
        const double* Wl = Wsp + (int64_t)l * N;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) w[4 * q + r] = Wl[tb_y<NT>(q, r, lane) * L + tb_x<NT>(q, lane)];
    };
    auto put = [&](int j, int q, int r, double v) {
        rows[(int64_t)(j - 1) * N + tb_y<NT>(q, r, lane) * L + tb_x<NT>(q, lane)] = v;
    };
    bool ok = true;
    double la_end;
    const double lz = dmfma_big_block_forward_end<NT>(
        Cb, L_tau, start, len, a, e, la, shift, wtab, put, [](int, int, double) {}, &la_end, &ok);
    if (lane == 0) {
        if (!ok) set_status(status, FH_ERR_NONFINITE, t.chain);
        blk_logz[c.blk_off + (int64_t)t.p * c.nb + t.block] = lz;
    }
}

// Two worldlines of the same (chain, spin, block) per wavefront: the W slice is shared and the
// two GEMM chains are independent, so one worldline's bf16 splitting, normalisation and stores
// overlap the other's matrix-core work. Same arithmetic as k_forward_mfma, step for step.
//
// Memory order. Vector loads and stores retire in issue order, so a wait for a load also waits
// for every store issued before it. The W slice of step j + 1 is therefore loaded before the
// stores of step j (a compiler fence keeps that order) and is waited for one step later, when
// those loads are long done and the stores may still be in flight. Task, chain, slice and row
// bases are wavefront-uniform (scalar registers), so a store is one lane offset plus a constant.
template <int LFIX>
__device__ __forceinline__ void forward_mfma2_body(
    int task, const ChainInfo* __restrict__ chains, const PairTask* __restrict__ tasks, int n_tasks,
    const uint16_t* __restrict__ cmat, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg, double* __restrict__ blk_la,
    float* __restrict__ endrow, const PairTask* __restrict__ ctasks,
    const int32_t* __restrict__ ccount) {
    const int lane = threadIdx.x & 63;
    // with the dense list of representative pairs (k_dedup), wavefront i takes its entry i
    if (task >= (ccount ? *ccount : n_tasks)) return;  // whole wavefront; no barriers here
    const PairTask t = ccount ? ctasks[task] : tasks[task];
    if (rescue_held(rsc, t.chain)) return;  // re-filtered whole in FP64 this pass
    const ChainInfo& c = chains[t.chain];
    // shared forward filters: only representatives run the recursion (k_member_logz completes
    // the others' log Z from the representative's end tile)
    const bool ra = !c.dedup || row_owner(rsc, c, t.p_a, t.block) == t.p_a;
    const bool rb = t.p_b >= 0 && (!c.dedup || row_owner(rsc, c, t.p_b, t.block) == t.p_b);
    if (!ra && !rb) return;
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const int L = LFIX ? LFIX : c.L, N = LFIX ? LFIX * LFIX : c.N, L_tau = c.L_tau;
    // a chain with few representatives (this pass's count from k_dedup) keeps its rows in the
    // cache for the members that read them next; otherwise the rows stream past it
    const int n_rep = c.dedup ? rsc.words[kRescueChain + 3 * rsc.n_chains + t.chain] : 0;
    const bool cached = n_rep > 0 && (int64_t)n_rep * (c.B - 1) * N * 4 <= kCachedRowBytes;
    const bool has_b = ra && rb;
    const int q0 = ra ? t.p_a : t.p_b;
    const int pp[2] = {q0, has_b ? t.p_b : q0};  // a lone worldline runs alone (PAIR false)
    const int spin = t.p_a >= c.n_up ? 1 : 0;
    const float* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const double coef = spin ? c.coef_dn : c.coef_up;
    const int32_t* pc = paths + c.path_off;
    int a[2], e[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        a[k] = pc[(int64_t)start * c.np + pp[k]];
        const int qe = start + len >= L_tau ? perm[c.part_off + pp[k]] : pp[k];  // reconnection
        e[k] = pc[(int64_t)((start + len) % L_tau) * c.np + qe];
        if (a[k] < 0 || a[k] >= N || e[k] < 0 || e[k] >= N) {
            if (lane == 0) set_status(status, FH_ERR_BAD_PATH, t.chain);
            a[k] = (a[k] < 0 || a[k] >= N) ? 0 : a[k];
            e[k] = (e[k] < 0 || e[k] >= N) ? 0 : e[k];
        }
    }
    Split3 C;
    {
        const uint4* cm = (const uint4*)(cmat + (size_t)t.chain * 3 * 2 * 64 * 8);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            C.h[q] = __builtin_bit_cast(bf16x8, cm[(0 * 2 + q) * 64 + lane]);
            C.m[q] = __builtin_bit_cast(bf16x8, cm[(1 * 2 + q) * 64 + lane]);
            C.l[q] = __builtin_bit_cast(bf16x8, cm[(2 * 2 + q) * 64 + lane]);
        }
    }
    const int x = lane & 31;
    const bool xin = LFIX ? true : x < L;
    // element (tile_row(lane, v), x) sits at lane_off + vrow(v) * L of a row
    const int lane_off = 4 * (lane >> 5) * L + x;
    auto vrow = [](int v) { return 8 * (v >> 2) + (v & 3); };
    auto inside = [&](int v) { return LFIX ? true : (xin && 4 * (lane >> 5) + vrow(v) < L); };
    auto load_w = [&](int l, float (&dst)[16]) {
        const float* Wl = Wsp + (int64_t)l * N;
        // a padded position reads site 0 (in bounds) and multiplies an exact zero of C f C
#pragma unroll
        for (int v = 0; v < 16; ++v) dst[v] = Wl[inside(v) ? lane_off + vrow(v) * L : 0];
    };
    // rows hold f~ 2^row_exp (the FP32 range scaling), from f_0 = 2^row_exp delta_a on
    const float sc = ldexpf(1.0f, c.row_exp);
    const double lsc = c.row_exp * 0.69314718055994530942;
    const float step_floor = c.step_floor;  // held in a register across the recursion
    // PAIR: two worldlines share the wavefront; a lone worldline (a representative without a
    // partner of its spin and block, the rule on a clustered state) runs alone, with half the
    // matrix and vector work per step, and the same arithmetic
    auto run = [&](auto pair) {
        constexpr bool PAIR = decltype(pair)::value;
        f32x16 F0, F1;
        {
            const int ax0 = a[0] % L, ay0 = a[0] / L, ax1 = a[1] % L, ay1 = a[1] / L;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int y = tile_row(lane, v);
                F0[v] = (x == ax0 && y == ay0) ? sc : 0.0f;
                if constexpr (PAIR) F1[v] = (x == ax1 && y == ay1) ? sc : 0.0f;
            }
        }
        double la0 = coef * (double)aux[c.aux_off + (int64_t)start * N + a[0]] - lsc;
        double la1 = PAIR ? coef * (double)aux[c.aux_off + (int64_t)start * N + a[1]] - lsc : 0.0;
        double prod0 = 1.0, prod1 = 1.0;
        const int64_t rowoff = (int64_t)t.block * (c.B - 1);
        float* rows0 = filt + c.filt_off + ((int64_t)pp[0] * L_tau + rowoff) * N;
        float* rows1 = filt + c.filt_off + ((int64_t)pp[1] * L_tau + rowoff) * N;
        // W of the current slice and of the next two, in three buffers that rotate every step:
        // a slice is loaded two steps before its use, so its load latency (longer than a step)
        // is hidden; with a single buffer the loop's back edge would copy the freshly loaded
        // slice into it and wait for the load in every step
        float wa[16], wb[16], wc[16];
        load_w((start + 1) % L_tau, wa);
        load_w((start + 2) % L_tau, wb);
        bool low0 = false, low1 = false;  // a worldline left FP32's range: FP64 re-filter
        // One step: uses wn (this slice's W) and loads the W of the slice after next into wf
        // before the stores, so that the wait before a W multiply leaves the stores in flight.
        auto step = [&](int j, const float (&wn)[16], float (&wf)[16]) {
            const int l = (start + j) % L_tau;
            f32x16 H0, H1;
            {
                const f32x16 X0 = circ_step(F0, C, neg);
                f32x16 X1;
                if constexpr (PAIR) X1 = circ_step(F1, C, neg);
                H0 = circ_step(X0, C, neg);
                if constexpr (PAIR) H1 = circ_step(X1, C, neg);
            }
            float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                F0[v] = H0[v] * wn[v];
                s0 += F0[v];
                if constexpr (PAIR) {
                    F1[v] = H1[v] * wn[v];
                    s1 += F1[v];
                }
            }
            // the W of the slice after next (the last two steps fetch slices they do not use;
            // always in bounds)
            load_w((l + 2) % L_tau, wf);
            __builtin_amdgcn_sched_barrier(0);
            const float tot0 = wave_sum_f32(s0), tot1 = PAIR ? wave_sum_f32(s1) : 1.0f;
            low0 |= !(tot0 >= step_floor) | !isfinite(tot0);
            if constexpr (PAIR) low1 |= !(tot1 >= step_floor) | !isfinite(tot1);
            // f~_j = h_j * inv: the normaliser applied is exactly 1/inv (see k_forward_mfma)
            const float inv0 = __builtin_amdgcn_rcpf(tot0);
            const float inv1 = PAIR ? __builtin_amdgcn_rcpf(tot1) : 1.0f;
            prod0 *= (double)inv0;
            if (!(prod0 > 1e-200 && prod0 < 1e200)) {
                la0 -= log(prod0);
                prod0 = 1.0;
            }
            if constexpr (PAIR) {
                prod1 *= (double)inv1;
                if (!(prod1 > 1e-200 && prod1 < 1e200)) {
                    la1 -= log(prod1);
                    prod1 = 1.0;
                }
            }
            const float k0 = inv0 * sc, k1 = inv1 * sc;
            float* row0 = rows0 + (int64_t)(j - 1) * N + lane_off;
            float* row1 = rows1 + (int64_t)(j - 1) * N + lane_off;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                F0[v] *= k0;
                if constexpr (PAIR) F1[v] *= k1;
                if (inside(v)) {
                    if (cached) {
                        row0[vrow(v) * L] = F0[v];
                        if constexpr (PAIR) row1[vrow(v) * L] = F1[v];
                    } else {
                        __builtin_nontemporal_store(F0[v], row0 + vrow(v) * L);
                        if constexpr (PAIR) __builtin_nontemporal_store(F1[v], row1 + vrow(v) * L);
                    }
                }
            }
        };
        if (len > 1) {
            step(1, wa, wc);
            int j = 2;
            for (; j + 2 < len; j += 3) {
                step(j, wb, wa);
                step(j + 1, wc, wb);
                step(j + 2, wa, wc);
            }
            if (j < len) step(j, wb, wa);
            if (j + 1 < len) step(j + 1, wc, wb);
        }
        {
            const double ms = block_shift_sum(shift, start, len, L_tau, lsc, lane);
            la0 += ms;
            la1 += ms;
        }
        // end weights (C f~ C)(e)
        f32x16 H0, H1;
        {
            const f32x16 X0 = circ_step(F0, C, neg);
            f32x16 X1;
            if constexpr (PAIR) X1 = circ_step(F1, C, neg);
            H0 = circ_step(X0, C, neg);
            if constexpr (PAIR) H1 = circ_step(X1, C, neg);
        }
        float hv0 = 0.0f, hv1 = 0.0f;
        {
            const int ex0 = e[0] % L, ey0 = e[0] / L, ex1 = e[1] % L, ey1 = e[1] / L;
            const int ve0 = (ey0 >> 3) * 4 + (ey0 & 3), ve1 = (ey1 >> 3) * 4 + (ey1 & 3);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                if (v == ve0) hv0 = H0[v];
                if constexpr (PAIR)
                    if (v == ve1) hv1 = H1[v];
            }
            hv0 = __shfl(hv0, ex0 + 32 * ((ey0 >> 2) & 1), 64);
            if constexpr (PAIR) hv1 = __shfl(hv1, ex1 + 32 * ((ey1 >> 2) & 1), 64);
        }
        la0 -= log(prod0);
        if constexpr (PAIR) la1 -= log(prod1);
        if (lane == 0) {
            if (low0 || !(hv0 >= kRangeFloor))
                rescue_push(rsc, c, t.chain, pp[0], t.block, low0 ? kCauseStep : kCauseEnd);
            blk_logz[c.blk_off + (int64_t)pp[0] * c.nb + t.block] = la0 + log((double)hv0);
            if constexpr (PAIR) {
                if (low1 || !(hv1 >= kRangeFloor))
                    rescue_push(rsc, c, t.chain, pp[1], t.block, low1 ? kCauseStep : kCauseEnd);
                blk_logz[c.blk_off + (int64_t)pp[1] * c.nb + t.block] = la1 + log((double)hv1);
            }
        }
        if (c.dedup) {  // what the worldlines sharing these rows need: log Z so far, end tile
            if (lane == 0) {
                blk_la[c.blk_off + (int64_t)pp[0] * c.nb + t.block] = la0;
                if constexpr (PAIR) blk_la[c.blk_off + (int64_t)pp[1] * c.nb + t.block] = la1;
            }
            float* end0 = endrow + c.end_off + ((int64_t)pp[0] * c.nb + t.block) * N + lane_off;
            float* end1 = endrow + c.end_off + ((int64_t)pp[1] * c.nb + t.block) * N + lane_off;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                if (inside(v)) {
                    end0[vrow(v) * L] = H0[v];
                    if constexpr (PAIR) end1[vrow(v) * L] = H1[v];
                }
            }
        }
    };
    if (has_b)
        run(std::true_type{});
    else
        run(std::false_type{});
}

template <int LFIX>
__global__ __launch_bounds__(kThreads, 2) void k_forward_mfma2(
    const ChainInfo* __restrict__ chains, const PairTask* __restrict__ tasks, int n_tasks,
    const uint16_t* __restrict__ cmat, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg, double* __restrict__ blk_la,
    float* __restrict__ endrow, const PairTask* __restrict__ ctasks,
    const int32_t* __restrict__ ccount) {
    // With the dense list the grid has kXcds spare workgroups. Phase A's FP64 recursions
    // (k_rescue_share_fwd4, one workgroup per representative, the first ones of their launch)
    // run beside this pass; workgroups are dealt to the XCDs in turn, so leaving as many leading
    // workgroups empty as there are such representatives (when fewer than kXcds) keeps this
    // pass's recursions off their XCDs, where a wavefront of each on one SIMD would share its
    // matrix core.
    int b = blockIdx.x;
    if (ccount) {
        const int n_a = rsc.words ? rsc.words[6] : 0;
        b -= n_a < kXcds ? n_a : 0;
        if (b < 0) return;
    }
    forward_mfma2_body<LFIX>(
        __builtin_amdgcn_readfirstlane(b * kWaves + (threadIdx.x >> 6)), chains, tasks,
        n_tasks, cmat, aux, W, wshift, aux_elems, total_slices, paths, perm, filt, blk_logz,
        sweep_ptr, status, rsc, neg, blk_la, endrow, ctasks, ccount);
}

// L = 64 on the same matrix cores: the 64 x 64 filter in four 32 x 32 sub-tiles X_RS (rows
// 32 R .., columns 32 S ..), each in the accumulator layout. X^T C is assembled from the
// sub-tile products of circ_step: (X^T C)_IJ = sum_K X_KI^T C_KJ, K in order, each term the six
// split products of the two K chunks. For L = 64 the circulant g((i - j) mod 64) has two
// distinct 32 x 32 blocks: C_00 = C_11 (T0) and C_01 = C_10 (T1, since -32 = 32 mod 64), so the
// operand holds two split blocks. Same arithmetic per product as the 32 x 32 tile: every
// product positive, FP32 accumulation, filters within the same bound.
// PAD (32 < L < 64, zero-padded to 64): the four blocks C_KJ differ (T[2 K + J]), each the
// circulant g((k - j) mod L) restricted to k, j < L.
template <bool PAD>
__device__ inline void circ64_step(const f32x16 (&X)[2][2], f32x16 (&Y)[2][2],
                                   const Split3 (&T)[PAD ? 4 : 2], const NegPairs& n) {
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
        for (int J = 0; J < 2; ++J) Y[I][J] = f32x16{};
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
        for (int K = 0; K < 2; ++K)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                bf16x8 h, m, l;
                split3_chunk(X[K][I], q, h, m, l, n);
#pragma unroll
                for (int J = 0; J < 2; ++J) {
                    const Split3& C = T[PAD ? 2 * K + J : (K == J ? 0 : 1)];
                    f32x16 acc = Y[I][J];
                    acc = mfma(l, C.h[q], acc);
                    acc = mfma(m, C.m[q], acc);
                    acc = mfma(m, C.h[q], acc);
                    acc = mfma(h, C.l[q], acc);
                    acc = mfma(h, C.m[q], acc);
                    acc = mfma(h, C.h[q], acc);
                    Y[I][J] = acc;
                }
            }
}

// The forward recursion of k_forward_mfma for L = 64 chains, one wavefront per (chain,
// worldline, block); rows stored as 4096 FP32 values, log Z as in k_forward_mfma. PAD: the
// chains with 32 < L < 64 on the same four sub-tiles, zero-padded to 64 x 64 (the padding stays
// an exact zero: C is zero outside L x L), with the four distinct operand blocks.
template <bool PAD>
__global__ __launch_bounds__(kThreads) void k_forward_mfma64(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const uint16_t* __restrict__ cmatb, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg) {
    constexpr int NB = PAD ? 4 : 2;  // operand blocks
    const int lane = threadIdx.x & 63;
    const int task = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    if (task >= n_tasks) return;  // whole wavefront; no barriers in this kernel
    const DrawTask t = tasks[task];
    const ChainInfo& c = chains[t.chain];
    // re-filtered whole in FP64 this pass (lattices with the FP64 circulant)
    if ((!PAD || fp64_circulant(c.L)) && rescue_held(rsc, t.chain)) return;
    const int L = PAD ? c.L : 64, N = PAD ? c.N : 4096;
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const int L_tau = c.L_tau;
    const int spin = t.p >= c.n_up ? 1 : 0;
    const float* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const double coef = spin ? c.coef_dn : c.coef_up;
    const int32_t* pc = paths + c.path_off;
    int a = pc[(int64_t)start * c.np + t.p];
    const int qe = start + len >= L_tau ? perm[c.part_off + t.p] : t.p;  // reconnection
    int e = pc[(int64_t)((start + len) % L_tau) * c.np + qe];
    if (a < 0 || a >= N || e < 0 || e >= N) {
        if (lane == 0) set_status(status, FH_ERR_BAD_PATH, t.chain);
        a = (a < 0 || a >= N) ? 0 : a;
        e = (e < 0 || e >= N) ? 0 : e;
    }
    Split3 T[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const uint4* cm = (const uint4*)(cmatb + ((size_t)t.chain * 4 + b) * 3 * 2 * 64 * 8);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            T[b].h[q] = __builtin_bit_cast(bf16x8, cm[(0 * 2 + q) * 64 + lane]);
            T[b].m[q] = __builtin_bit_cast(bf16x8, cm[(1 * 2 + q) * 64 + lane]);
            T[b].l[q] = __builtin_bit_cast(bf16x8, cm[(2 * 2 + q) * 64 + lane]);
        }
    }
    const int x = lane & 31;
    // element (32 R + tile_row(lane, v), 32 S + x) of sub-tile (R, S) sits at
    // lane_off + 32 (R L + S) + vrow(v) L of a row
    const int lane_off = 4 * (lane >> 5) * L + x;
    auto vrow = [](int v) { return 8 * (v >> 2) + (v & 3); };
    auto inside = [&](int R, int S, int v) {
        return !PAD || (32 * S + x < L && 32 * R + 4 * (lane >> 5) + vrow(v) < L);
    };
    auto load_w = [&](int l, float (&dst)[2][2][16]) {
        const float* Wl = Wsp + (int64_t)l * N;
        // a padded position reads the slice's first site and multiplies an exact zero
#pragma unroll
        for (int R = 0; R < 2; ++R)
#pragma unroll
            for (int S = 0; S < 2; ++S)
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    dst[R][S][v] =
                        Wl[inside(R, S, v) ? lane_off + 32 * (R * L + S) + vrow(v) * L : 0];
    };
    // rows hold f~ 2^row_exp (the FP32 range scaling), from f_0 = 2^row_exp delta_a on
    const float sc = ldexpf(1.0f, c.row_exp);
    const double lsc = c.row_exp * 0.69314718055994530942;
    const float step_floor = c.step_floor;  // held in a register across the recursion
    f32x16 F[2][2];
    {
        const int ax = a % L, ay = a / L;
#pragma unroll
        for (int R = 0; R < 2; ++R)
#pragma unroll
            for (int S = 0; S < 2; ++S)
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    F[R][S][v] = (32 * S + x == ax && 32 * R + tile_row(lane, v) == ay) ? sc : 0.0f;
    }
    double la = coef * (double)aux[c.aux_off + (int64_t)start * N + a] - lsc;
    double prod = 1.0;
    float* rows = filt + c.filt_off + ((int64_t)t.p * L_tau + (int64_t)t.block * (c.B - 1)) * N;
    // W of the next slice is loaded before this slice's stores (loads and stores retire in
    // order), so its wait one step later does not wait for them; the padded variant, whose four
    // operand blocks take the registers of that prefetch, loads it between the two products
    float wn[2][2][16];
    if constexpr (!PAD) load_w((start + 1) % L_tau, wn);
    bool low = false;  // the block left FP32's range (the FP64 re-filter takes L <= 32 only)
    for (int j = 1; j < len; ++j) {
        const int l = (start + j) % L_tau;
        f32x16 X[2][2], H[2][2];
        circ64_step<PAD>(F, X, T, neg);
        if constexpr (PAD) load_w(l, wn);  // in flight during the second product
        circ64_step<PAD>(X, H, T, neg);
        float s = 0.0f;
#pragma unroll
        for (int R = 0; R < 2; ++R)
#pragma unroll
            for (int S = 0; S < 2; ++S)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    F[R][S][v] = H[R][S][v] * wn[R][S][v];
                    s += F[R][S][v];
                }
        if constexpr (!PAD) load_w((l + 1) % L_tau, wn);  // the last step fetches a slice it does not use
        __builtin_amdgcn_sched_barrier(0);
        const float tot = wave_sum_f32(s);
        low |= !(tot >= step_floor) | !isfinite(tot);
        // f~_j = h_j * inv: the normaliser applied is exactly 1/inv (see k_forward_mfma)
        const float inv = __builtin_amdgcn_rcpf(tot);
        prod *= (double)inv;
        if (!(prod > 1e-200 && prod < 1e200)) {
            la -= log(prod);
            prod = 1.0;
        }
        const float k = inv * sc;
        float* row = rows + (int64_t)(j - 1) * N + lane_off;
#pragma unroll
        for (int R = 0; R < 2; ++R)
#pragma unroll
            for (int S = 0; S < 2; ++S)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    F[R][S][v] *= k;
                    if (inside(R, S, v))
                        __builtin_nontemporal_store(F[R][S][v], row + 32 * (R * L + S) + vrow(v) * L);
                }
    }
    la += block_shift_sum(shift, start, len, L_tau, lsc, lane);
    // end weight (C f~ C)(e)
    f32x16 X[2][2], H[2][2];
    circ64_step<PAD>(F, X, T, neg);
    circ64_step<PAD>(X, H, T, neg);
    const int ex = e % L, ey = e / L;
    const int Re = ey >> 5, Se = ex >> 5, ty = ey & 31, tx = ex & 31;
    const int ve = (ty >> 3) * 4 + (ty & 3);
    float hv = 0.0f;
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int S = 0; S < 2; ++S)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                if (R == Re && S == Se && v == ve) hv = H[R][S][v];
    hv = __shfl(hv, tx + 32 * ((ty >> 2) & 1), 64);
    la -= log(prod);
    if (lane == 0) {
        if (low || !(hv >= kRangeFloor))
            rescue_push(rsc, c, t.chain, t.p, t.block, low ? kCauseStep : kCauseEnd);
        blk_logz[c.blk_off + (int64_t)t.p * c.nb + t.block] = la + log((double)hv);
    }
}

// Raw buffer resources: word 3 of the descriptor on gfx9-family chips (32-bit data format,
// no swizzle), and the cache-policy bit of a streaming (nontemporal) store.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kNontemporal = 2;

// Bits of a float for the b32 buffer store. The value is taken as a function argument: applied
// directly to an element of an ext_vector_type, __builtin_bit_cast reads element 0 whatever the
// index (seen with this compiler), so it never gets a vector element.
__device__ inline uint32_t fbits(float f) { return __builtin_bit_cast(uint32_t, f); }

// Segmented sum over the lanes that share a column block of BS lanes (BS = 16: the DPP rows
// J and J + 2; BS = 8: the half rows J and J + 4): every lane gets its block's sum. The two
// halves of the wavefront meet through v_permlane32_swap, which exchanges one half of its
// destination with the other half of its source: the two results hold the low half's values
// in one and the high half's in the other, so their sum is the same in every lane.
template <int BS>
__device__ inline float block_sum(float v) {
    v = dpp_add<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141>(v);  // row_half_mirror: sums over 8 lanes
    if (BS == 16) v = dpp_add<0x140>(v);  // row_mirror: sums over 16 lanes
    // both halves of the wavefront, in the same operand order in every lane
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, v),
                                                    __builtin_bit_cast(uint32_t, v), false, false);
    return __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
}

// Small lattices packed block-diagonally (L <= BS = 32 / P). P x P worldlines of one (chain,
// spin, block) share a 32 x 32 tile: worldline (I, J) of the tile occupies rows BS I .. BS I + L - 1
// and columns BS J .. BS J + L - 1, and the circulant operand is block-diagonal with one L x L
// circulant g((i - j) mod L) per diagonal block. Every term coupling two blocks is an exact zero,
// so C F C is C_L F_IJ C_L block by block, with the same six split products as the padded tile
// of k_forward_mfma: same arithmetic, P^2 worldlines for the matrix work of one. NT tiles per
// wavefront (two tiles overlap one tile's splitting with the other's matrix work, as in
// k_forward_mfma2; one tile doubles the wavefronts of a small batch).
//
// Slots. Slot s = T P^2 + I P + J (tile T, block (I, J)) of a task holds worldline
// wl(min(s, n - 1)), wl(k) = p0 + k; slots past n repeat the last worldline and are neither
// stored nor counted. Each block's normaliser comes from a segmented wavefront sum; the slot's
// log Z is kept by its owner lane BS J + T P + I (first half of the wavefront) as an FP64
// mantissa and a binary exponent, renormalised every step, so no log is taken inside the loop.
// Shared forward filters: with the dense list of tiles of representatives (k_dedup), wavefront
// i takes its entry i and wl(k) = prep[p0 + k]; each representative also leaves its log Z before
// the end weight and its end tile for the worldlines that share its rows (k_member_logz). A
// worldline's arithmetic does not depend on its slot: the other blocks contribute exact zeros,
// and every block sums its terms in the same order.
template <int P, int NT>
__device__ __forceinline__ void forward_pack_body(
    int task, const ChainInfo* __restrict__ chains, const PackTask* __restrict__ tasks, int n_tasks,
    const uint16_t* __restrict__ cmatp, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg, double* __restrict__ blk_la,
    float* __restrict__ endrow, const PackTask* __restrict__ ctasks,
    const int32_t* __restrict__ ccount, const int32_t* __restrict__ prep) {
    constexpr int BS = 32 / P;   // block side
    constexpr int PP = P * P;    // worldlines per tile
    constexpr int RPB = 16 / P;  // registers of one block row band per lane
    const int lane = threadIdx.x & 63;
    if (task >= (ccount ? *ccount : n_tasks)) return;  // whole wavefront; no barriers here
    const PackTask t = ccount ? ctasks[task] : tasks[task];
    if (rescue_held(rsc, t.chain)) return;  // re-filtered whole in FP64 this pass
    const ChainInfo& c = chains[t.chain];
    auto wl = [&](int k) { return ccount ? prep[t.p0 + k] : t.p0 + k; };
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const int L = c.L, N = c.N, L_tau = c.L_tau;
    const int spin = wl(0) >= c.n_up ? 1 : 0;
    const float* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const double coef = spin ? c.coef_dn : c.coef_up;
    const int32_t* pc = paths + c.path_off;
    // a full task (every slot its own worldline, L filling the blocks) stores unmasked
    const bool full = t.n == NT * PP && L == BS;

    Split3 C;
    {
        const uint4* cm = (const uint4*)(cmatp + (size_t)t.chain * 3 * 2 * 64 * 8);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            C.h[q] = __builtin_bit_cast(bf16x8, cm[(0 * 2 + q) * 64 + lane]);
            C.m[q] = __builtin_bit_cast(bf16x8, cm[(1 * 2 + q) * 64 + lane]);
            C.l[q] = __builtin_bit_cast(bf16x8, cm[(2 * 2 + q) * 64 + lane]);
        }
    }
    const int x = lane & 31, hl = lane >> 5;
    const int J = x / BS, lx = x % BS;
    // register v holds tile row 8 (v / 4) + 4 hl + v % 4: block row I(v) = v / RPB, local row
    // 4 hl + cv(v)
    auto cv = [](int v) { return 8 * (v >> 2) + (v & 3) - BS * (v / RPB); };
    const int64_t rowoff = (int64_t)t.block * (c.B - 1);
    // per (tile, block row): this lane's slot, its byte offset in the chain's filter region
    // (element (4 hl + cv(v), lx) of the block at off + 4 cv(v) L) and whether it is stored.
    // The region is addressed through a buffer resource (32-bit offsets; the plan packs only
    // chains whose filter region is under 2 GiB).
    const __amdgpu_buffer_rsrc_t frs = __builtin_amdgcn_make_buffer_rsrc(
        filt + c.filt_off, (short)0, 0x7fffffff, kBufferWord3);
    uint32_t off[NT][P];
    bool ok[NT][P];
    // rows hold f~ 2^row_exp (the FP32 range scaling), from f_0 = 2^row_exp delta_a on
    const float sc = ldexpf(1.0f, c.row_exp);
    const double lsc = c.row_exp * 0.69314718055994530942;
    const float step_floor = c.step_floor;  // held in a register across the recursion
    f32x16 F[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T)
#pragma unroll
        for (int I = 0; I < P; ++I) {
            const int s = T * PP + I * P + J;
            const int pw = wl(s < t.n ? s : t.n - 1);
            int a = pc[(int64_t)start * c.np + pw];
            a = (a < 0 || a >= N) ? 0 : a;  // reported by the owner lane below
            const int ax = a % L, ay = a / L;
#pragma unroll
            for (int v = I * RPB; v < (I + 1) * RPB; ++v)
                F[T][v] = (lx == ax && 4 * hl + cv(v) == ay) ? sc : 0.0f;
            off[T][I] = (uint32_t)((((int64_t)pw * L_tau + rowoff) * N + 4 * hl * L + lx) * 4);
            ok[T][I] = s < t.n && lx < L;
        }
    // owner lane: slot (T, I, J) with T P + I = lx, first half
    const int oti = lx;
    const int oT = oti / P, oI = oti % P;
    const int os = oT * PP + oI * P + J;
    const bool owner = hl == 0 && oti < NT * P && os < t.n;
    int oe = 0;
    double la = 0.0, mant = 1.0;
    int ex2 = 0;
    const int opw = owner ? wl(os) : 0;
    if (owner) {
        const int pw = opw;
        const int a = pc[(int64_t)start * c.np + pw];
        const int qe = start + len >= L_tau ? perm[c.part_off + pw] : pw;  // reconnection
        oe = pc[(int64_t)((start + len) % L_tau) * c.np + qe];
        if (a < 0 || a >= N || oe < 0 || oe >= N) {
            set_status(status, FH_ERR_BAD_PATH, t.chain);
            oe = (oe < 0 || oe >= N) ? 0 : oe;
        } else {
            la = coef * (double)aux[c.aux_off + (int64_t)start * N + a] - lsc;
        }
    }
    auto inside = [&](int v) { return lx < L && 4 * hl + cv(v) < L; };
    auto load_w = [&](int l, float (&dst)[16]) {
        const float* Wl = Wsp + (int64_t)l * N + 4 * hl * L + lx;
        // a padded position reads the slice's first site and multiplies an exact zero of C f C
#pragma unroll
        for (int v = 0; v < 16; ++v) dst[v] = inside(v) ? Wl[cv(v) * L] : Wsp[(int64_t)l * N];
    };
    bool low = false;  // the owner's worldline left FP32's range: FP64 re-filter
    // two W buffers that swap roles every step (one buffer would make the loop's back edge copy
    // the loaded slice into it, waiting for the load)
    float wa[16], wb[16];
    load_w((start + 1) % L_tau, wa);
    auto step = [&](int j, const float (&wn)[16], float (&wf)[16]) {
        const int l = (start + j) % L_tau;
        f32x16 H[NT];
#pragma unroll
        for (int T = 0; T < NT; ++T) H[T] = circ_step(F[T], C, neg);
#pragma unroll
        for (int T = 0; T < NT; ++T) H[T] = circ_step(H[T], C, neg);
        float sm[NT][P];
#pragma unroll
        for (int T = 0; T < NT; ++T)
#pragma unroll
            for (int I = 0; I < P; ++I) sm[T][I] = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v)
#pragma unroll
            for (int T = 0; T < NT; ++T) {
                F[T][v] = H[T][v] * wn[v];
                sm[T][v / RPB] += F[T][v];
            }
        load_w((l + 1) % L_tau, wf);  // the last step fetches a slice it does not use
        __builtin_amdgcn_sched_barrier(0);
        float inv[NT][P], mine = 1.0f, mtot = 1.0f;
#pragma unroll
        for (int T = 0; T < NT; ++T)
#pragma unroll
            for (int I = 0; I < P; ++I) {
                const float tot = block_sum<BS>(sm[T][I]);
                // f~_j = h_j * inv: the normaliser applied is exactly 1/inv
                inv[T][I] = __builtin_amdgcn_rcpf(tot);
                mine = oti == T * P + I ? inv[T][I] : mine;
                mtot = oti == T * P + I ? tot : mtot;
            }
        low |= !(mtot >= step_floor && mtot <= 3.402823466e38f);
        // log Z -= log(inv): FP64 mantissa times 2^ex2, renormalised every step
        mant *= (double)mine;
        int e;
        mant = frexp(mant, &e);
        ex2 += e;
        // byte offsets: lane part in a VGPR, row and register part in an SGPR
        const int rowj = (j - 1) * N;
#pragma unroll
        for (int v = 0; v < 16; ++v)
#pragma unroll
            for (int T = 0; T < NT; ++T) F[T][v] *= inv[T][v / RPB] * sc;
        if (full) {
#pragma unroll
            for (int v = 0; v < 16; ++v)
#pragma unroll
                for (int T = 0; T < NT; ++T)
                    __builtin_amdgcn_raw_buffer_store_b32(fbits(F[T][v]), frs, off[T][v / RPB],
                                                          (rowj + cv(v) * L) * 4, kNontemporal);
        } else {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const bool in = 4 * hl + cv(v) < L;
#pragma unroll
                for (int T = 0; T < NT; ++T)
                    if (in && ok[T][v / RPB])
                        __builtin_amdgcn_raw_buffer_store_b32(fbits(F[T][v]), frs, off[T][v / RPB],
                                                              (rowj + cv(v) * L) * 4, kNontemporal);
            }
        }
    };
    if (len > 1) {
        step(1, wa, wb);
        int j = 2;
        for (; j + 1 < len; j += 2) {
            step(j, wb, wa);
            step(j + 1, wa, wb);
        }
        if (j < len) step(j, wb, wa);
    }
    la += block_shift_sum(shift, start, len, L_tau, lsc, lane);
    // end weights (C f~ C)(e) of every slot: the owner reads its block's element at e
    f32x16 H[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T) H[T] = circ_step(circ_step(F[T], C, neg), C, neg);
    const int row = BS * oI + oe / L, col = BS * J + oe % L;
    const int src = col + 32 * ((row >> 2) & 1), ve = 4 * (row >> 3) + (row & 3);
    float hv = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v)
#pragma unroll
        for (int T = 0; T < NT; ++T) {
            const float h = __shfl(H[T][v], src, 64);
            if (v == ve && T == oT) hv = h;
        }
    const double la_end = la - (log(mant) + (double)ex2 * 0.69314718055994530942);
    if (owner) {
        if (low || !(hv >= kRangeFloor))
            rescue_push(rsc, c, t.chain, opw, t.block, low ? kCauseStep : kCauseEnd);
        blk_logz[c.blk_off + (int64_t)opw * c.nb + t.block] = la_end + log((double)hv);
        if (c.dedup) blk_la[c.blk_off + (int64_t)opw * c.nb + t.block] = la_end;
    }
    if (c.dedup) {  // the end tiles of the slots, for the worldlines that share their rows
#pragma unroll
        for (int T = 0; T < NT; ++T)
#pragma unroll
            for (int I = 0; I < P; ++I) {
                const int s = T * PP + I * P + J;
                if (!ok[T][I]) continue;
                float* end = endrow + c.end_off + ((int64_t)wl(s) * c.nb + t.block) * N +
                             4 * hl * L + lx;
#pragma unroll
                for (int v = I * RPB; v < (I + 1) * RPB; ++v)
                    if (4 * hl + cv(v) < L) end[cv(v) * L] = H[T][v];
            }
    }
}

template <int P, int NT>
__global__ __launch_bounds__(kThreads, NT == 1 ? 4 : 2) void k_forward_pack(
    const ChainInfo* __restrict__ chains, const PackTask* __restrict__ tasks, int n_tasks,
    const uint16_t* __restrict__ cmatp, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg, double* __restrict__ blk_la,
    float* __restrict__ endrow, const PackTask* __restrict__ ctasks,
    const int32_t* __restrict__ ccount, const int32_t* __restrict__ prep) {
    forward_pack_body<P, NT>(
        __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6)), chains, tasks,
        n_tasks, cmatp, aux, W, wshift, aux_elems, total_slices, paths, perm, filt, blk_logz,
        sweep_ptr, status, rsc, neg, blk_la, endrow, ctasks, ccount, prep);
}

// One step of the adjoint's ring recursion for one worldline per wavefront:
// F <- W~_l . (C F C) / total (W~ read from Wl, padded sites 0); returns 1 / total and sets
// *bad when the total is not a positive finite number. The forward pass and the checkpoint
// recompute share it, so the recomputed rows are the stored ones bit for bit.
template <int LFIX>
__device__ __forceinline__ float ring_step(f32x16& F, const float* Wl, const Split3& C,
                                           const NegPairs& neg, int lane, int L, bool* bad) {
    const int x = lane & 31;
    const bool xin = LFIX ? true : x < L;
    float w[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int y = tile_row(lane, v);
        const bool in = LFIX ? true : (xin && y < L);
        const float wv0 = Wl[in ? y * L + x : 0];
        w[v] = in ? wv0 : 0.0f;
    }
    __builtin_amdgcn_sched_barrier(0);  // W in flight during the matrix work
    const f32x16 X = circ_step(F, C, neg);
    const f32x16 H = circ_step(X, C, neg);
    float s = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        F[v] = H[v] * w[v];
        s += F[v];
    }
    const float tot = wave_sum_f32(s);
    *bad = !(tot > 0.0f) || !isfinite(tot);
    const float inv = __builtin_amdgcn_rcpf(tot);
#pragma unroll
    for (int v = 0; v < 16; ++v) F[v] *= inv;
    return inv;
}

template <int LFIX>
__device__ __forceinline__ void ring_store(float* row, const f32x16& F, int lane, int L) {
    const int x = lane & 31;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int y = tile_row(lane, v);
        if (LFIX || (x < L && y < L)) row[y * L + x] = F[v];
    }
}

// Adjoint of the forward filter over the ring anchored at `anchor` (one block of length L_tau,
// closing on the anchor site e of the reconnected worldline, e = a without reconnection), on
// the matrix cores. A workgroup takes up to kGroup worldlines of one (chain, spin), one per
// wavefront, in lockstep over the slices:
//   forward:  f~_j as in k_forward_mfma, every row j = 0..L_tau-1 stored (row 0 = delta_a)
//   backward: u_{L_tau} = delta_e; beta_j = C u_{j+1} C; u_j = W~_j . beta_j / sum
//   d log Z / d log W_j(r) = f~_j(r) beta_j(r) / <f~_j, beta_j>   (the smoothing marginal)
//   d log Z / d t += dtau <A beta_j, f~_j> / <beta_j, f~_j>, A the nearest-neighbour hopping
//                    matrix: G = exp(t dtau A), so dG/dt = dtau A G and <u, (dG/dt) f> =
//                    dtau <A G u, f>; A beta is a four-neighbour stencil read from LDS.
// The marginals of the group are summed in LDS and written (times the spin's coefficient) to
// the group's partial slab; k_gpart_reduce adds the slabs of a chain in a fixed order, so the
// field gradient is the same on every call.
// With ckpt (FH_FLAG_GRAD_CHECKPOINT) the forward pass keeps only rows j = 0, K, 2K, .. (K =
// ceil(sqrt(L_tau))); when the backward messages enter a segment sK .. sK + K - 1 from above,
// every wavefront recomputes rows sK + 1 .. of it from checkpoint s with the same steps, into
// its own K - 1 segment rows. The recomputed rows are bit-identical to the stored ones, so the
// gradient is the same with and without checkpoints; rows held drop from L_tau to about
// 2 sqrt(L_tau) per worldline, for one more forward recursion.
template <int LFIX, bool CK>
__global__ __launch_bounds__(kThreads, LFIX || !CK ? 3 : 2) void k_grad_mfma(
    const ChainInfo* __restrict__ chains, const GroupTask* __restrict__ groups,
    const uint16_t* __restrict__ cmat, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, float* __restrict__ filt, float* __restrict__ gpart,
    double* __restrict__ blk_logz, double* __restrict__ dt_out, int anchor,
    const int32_t* __restrict__ perm, int32_t* status, const NegPairs neg,
    float* __restrict__ ckpt) {
    // beta tile of each wavefront with a halo row on each side: row y at (y + 1) * 32, row -1
    // repeats row L - 1 and row L repeats row 0, so the four-neighbour stencil reads at fixed
    // offsets from three per-lane bases
    __shared__ float bt[kWaves][34 * 32];
    __shared__ float mg[2][kWaves][1024];  // marginal tiles, double-buffered over the slices
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const GroupTask g = groups[blockIdx.x];
    const ChainInfo& c = chains[g.chain];
    const int L = LFIX ? LFIX : c.L, N = LFIX ? LFIX * LFIX : c.N, L_tau = c.L_tau;
    const bool real = wv < g.count;            // extra wavefronts shadow worldline p0
    const int p = g.p0 + (real ? wv : 0);
    const float* Wsp = W + g.spin * aux_elems + c.aux_off;
    const double* shift = wshift + g.spin * total_slices + c.slice_off;
    const double coef = g.spin ? c.coef_dn : c.coef_up;
    const double dtau = c.dtau;
    int a = paths[c.path_off + (int64_t)anchor * c.np + p];
    // the ring closes on the anchor site of the reconnected worldline (itself for the identity)
    int e = paths[c.path_off + (int64_t)anchor * c.np + perm[c.part_off + p]];
    if (a < 0 || a >= N || e < 0 || e >= N) {
        if (lane == 0 && real) set_status(status, FH_ERR_BAD_PATH, g.chain);
        a = a < 0 || a >= N ? 0 : a;
        e = e < 0 || e >= N ? 0 : e;
    }
    Split3 C;
    {
        const uint4* cm = (const uint4*)(cmat + (size_t)g.chain * 3 * 2 * 64 * 8);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            C.h[q] = __builtin_bit_cast(bf16x8, cm[(0 * 2 + q) * 64 + lane]);
            C.m[q] = __builtin_bit_cast(bf16x8, cm[(1 * 2 + q) * 64 + lane]);
            C.l[q] = __builtin_bit_cast(bf16x8, cm[(2 * 2 + q) * 64 + lane]);
        }
    }
    const int x = lane & 31;
    const bool xin = LFIX ? true : x < L;
    const int ax = a % L, ay = a / L, ex = e % L, ey = e / L;
    float* rows = filt + c.filt_off + (int64_t)p * L_tau * N;
    constexpr bool ck = CK;  // ckpt is given exactly for CK
    const int K = ck ? c.ck_k : 1;
    float* ckrows = ck ? ckpt + c.ck_row_off + (int64_t)p * c.ck_n * N : nullptr;
    float* seg = ck ? ckpt + g.seg_off + (int64_t)wv * (K - 1) * N : nullptr;
    // ring row j: the filter workspace, or checkpoint j / K (j % K == 0) or row j % K - 1 of
    // this wavefront's segment
    auto ring_row = [&](int j) -> float* {
        if (!ck) return rows + (int64_t)j * N;
        const int sj = j / K, i = j - sj * K;
        return i == 0 ? ckrows + (int64_t)sj * N : seg + (int64_t)(i - 1) * N;
    };
    // ---- forward pass over the ring, every row (every K-th with checkpoints) stored
    f32x16 F;
#pragma unroll
    for (int v = 0; v < 16; ++v) F[v] = (x == ax && tile_row(lane, v) == ay) ? 1.0f : 0.0f;
    if (real) ring_store<LFIX>(ring_row(0), F, lane, L);
    double la = coef * (double)aux[c.aux_off + (int64_t)anchor * N + a];
    double prod = 1.0;
    for (int j = 1; j < L_tau; ++j) {
        const int l = (anchor + j) % L_tau;
        bool bad;
        const float inv = ring_step<LFIX>(F, Wsp + (int64_t)l * N, C, neg, lane, L, &bad);
        if (bad && real && lane == 0) set_status(status, FH_ERR_NONFINITE, g.chain);
        prod *= (double)inv;
        if (!(prod > 1e-200 && prod < 1e200)) {
            la -= log(prod);
            prod = 1.0;
        }
        la += shift[l];
        if (real && j % K == 0) ring_store<LFIX>(ring_row(j), F, lane, L);
    }
    {
        const f32x16 X = circ_step(F, C, neg);
        const f32x16 H = circ_step(X, C, neg);
        float hv = 0.0f;
        const int ve = (ey >> 3) * 4 + (ey & 3);
#pragma unroll
        for (int v = 0; v < 16; ++v)
            if (v == ve) hv = H[v];
        hv = __shfl(hv, ex + 32 * ((ey >> 2) & 1), 64);
        la -= log(prod);
        if (real && lane == 0) {
            if (!(hv > 0.0f)) set_status(status, FH_ERR_NONFINITE, g.chain);
            blk_logz[c.blk_off + (int64_t)p * c.nb] = la + log((double)hv);
        }
    }
    __syncthreads();  // every row of the group is stored before any wavefront reads one back
    // ---- backward messages
    f32x16 U;
#pragma unroll
    for (int v = 0; v < 16; ++v) U[v] = (x == ex && tile_row(lane, v) == ey) ? 1.0f : 0.0f;
    double dt = 0.0;
    float* slab = gpart + g.part_off;
    const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
    float* btw = bt[wv] + 4 * (lane >> 5) * 32;  // row 4 (lane / 32) - 1 of the halo layout
    for (int j = L_tau - 1; j >= 0; --j) {
        const int l = (anchor + j) % L_tau;
        if (ck && j % K != 0 && (j == L_tau - 1 || (j + 1) % K == 0)) {
            // entering segment j / K from above: its rows from the checkpoint, every wavefront
            // (shadows too) into its own segment rows
            const int j0 = j - j % K;
            const float* c0 = ring_row(j0);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int y = tile_row(lane, v);
                const bool in = LFIX ? true : (xin && y < L);
                const float f0 = c0[in ? y * L + x : 0];
                F[v] = in ? f0 : 0.0f;
            }
            for (int i = j0 + 1; i <= j; ++i) {
                bool bad;  // the forward pass reported it already
                ring_step<LFIX>(F, Wsp + (int64_t)((anchor + i) % L_tau) * N, C, neg, lane, L,
                                &bad);
                ring_store<LFIX>(ring_row(i), F, lane, L);
            }
        }
        // this slice's filter row and W: issued before the matrix work, waited for after it
        const float* row = ring_row(j);
        const float* Wl = Wsp + (int64_t)l * N;
        float fj[16], wl[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int y = tile_row(lane, v);
            const bool in = LFIX ? true : (xin && y < L);
            fj[v] = row[in ? y * L + x : 0];
            wl[v] = Wl[in ? y * L + x : 0];
        }
        __builtin_amdgcn_sched_barrier(0);
        const f32x16 X = circ_step(U, C, neg);
        const f32x16 B = circ_step(X, C, neg);   // beta_j = C u_{j+1} C
        float den = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int y = tile_row(lane, v);
            const bool in = LFIX ? true : (xin && y < L);
            fj[v] = in ? fj[v] : 0.0f;
            den += fj[v] * B[v];
            const float bv = in ? B[v] : 0.0f;
            const int r = 8 * (v >> 2) + (v & 3);  // y = 4 (lane / 32) + r
            // rows past L - 1 are not written: row L's slot holds the halo copy of row 0
            if (LFIX || y < L) btw[(r + 1) * 32 + x] = bv;
            if (y == L - 1) bt[wv][x] = bv;                 // halo row -1
            if (y == 0) bt[wv][(L + 1) * 32 + x] = bv;      // halo row L
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float num = 0.0f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int y = tile_row(lane, v);
            const bool in = LFIX ? true : (xin && y < L);
            const int r = 8 * (v >> 2) + (v & 3);
            const float nbr = btw[(r + 1) * 32 + xp] + btw[(r + 1) * 32 + xm] +
                              btw[(r + 2) * 32 + x] + btw[r * 32 + x];
            num += in ? fj[v] * nbr : 0.0f;
        }
        const double dden = (double)wave_sum_f32(den);
        const double dnum = (double)wave_sum_f32(num);
        dt += dtau * dnum / dden;
        const float k = real ? (float)(coef / dden) : 0.0f;
        float* mgb = mg[j & 1][wv];
#pragma unroll
        for (int v = 0; v < 16; ++v) mgb[tile_row(lane, v) * 32 + x] = k * fj[v] * B[v];
        __syncthreads();  // one barrier per slice: the tiles of slice j + 2 reuse these buffers
        {
            const float* m0 = mg[j & 1][0];
            const float* m1 = mg[j & 1][1];
            const float* m2 = mg[j & 1][2];
            const float* m3 = mg[j & 1][3];
            float* srow = slab + (int64_t)l * N;
            for (int i = threadIdx.x; i < 1024; i += kThreads) {
                const int yy = i >> 5, xx = i & 31;
                if (LFIX || (xx < L && yy < L)) srow[yy * L + xx] = (m0[i] + m1[i]) + (m2[i] + m3[i]);
            }
        }
        if (j > 0) {
            float s = 0.0f;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int y = tile_row(lane, v);
                const bool in = LFIX ? true : (xin && y < L);
                U[v] = in ? wl[v] * B[v] : 0.0f;
                s += U[v];
            }
            const float tot = wave_sum_f32(s);
            if ((!(tot > 0.0f) || !isfinite(tot)) && real && lane == 0)
                set_status(status, FH_ERR_NONFINITE, g.chain);
            const float inv = __builtin_amdgcn_rcpf(tot);
#pragma unroll
            for (int v = 0; v < 16; ++v) U[v] *= inv;
        }
    }
    if (real && lane == 0) dt_out[c.part_off + p] = dt;
}

// The adjoint of k_grad_mfma on the FP64 matrix cores (FP64 plans, every chain L <= 32): the
// same ring, recursion, marginals and d/dt stencil, every product and sum in FP64 with the
// circulant of k_forward_dmfma; ring rows stored as FP64 rows, group partial slabs in FP64;
// the checkpoints of FH_FLAG_GRAD_CHECKPOINT as in k_grad_mfma.
template <bool CK>
__global__ __launch_bounds__(kThreads) void k_grad_dmfma(
    const ChainInfo* __restrict__ chains, const GroupTask* __restrict__ groups,
    const double* __restrict__ cmat64, const double* __restrict__ aux,
    const double* __restrict__ W, const double* __restrict__ wshift, int64_t aux_elems,
    int64_t total_slices, const int32_t* __restrict__ paths, double* __restrict__ filt,
    double* __restrict__ gpart, double* __restrict__ blk_logz, double* __restrict__ dt_out,
    int anchor, const int32_t* __restrict__ perm, int32_t* status, double* __restrict__ ckpt) {
    // beta tile of each wavefront with halo rows (row y at (y + 1) * 32; row -1 repeats row L - 1,
    // row L repeats row 0), and double-buffered marginal tiles, as in k_grad_mfma
    __shared__ double bt[kWaves][34 * 32];
    __shared__ double mg[2][kWaves][1024];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const GroupTask g = groups[blockIdx.x];
    const ChainInfo& c = chains[g.chain];
    const int L = c.L, N = c.N, L_tau = c.L_tau;
    const bool real = wv < g.count;  // extra wavefronts shadow worldline p0
    const int p = g.p0 + (real ? wv : 0);
    const double* Wsp = W + g.spin * aux_elems + c.aux_off;
    const double* shift = wshift + g.spin * total_slices + c.slice_off;
    const double coef = g.spin ? c.coef_dn : c.coef_up;
    const double dtau = c.dtau;
    int a = paths[c.path_off + (int64_t)anchor * c.np + p];
    // the ring closes on the anchor site of the reconnected worldline (itself for the identity)
    int e = paths[c.path_off + (int64_t)anchor * c.np + perm[c.part_off + p]];
    if (a < 0 || a >= N || e < 0 || e >= N) {
        if (lane == 0 && real) set_status(status, FH_ERR_BAD_PATH, g.chain);
        a = a < 0 || a >= N ? 0 : a;
        e = e < 0 || e >= N ? 0 : e;
    }
    double Cb[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) Cb[q] = cmat64[((int64_t)g.chain * 16 + q) * 64 + lane];
    const int xl = lane & 15, yl = lane >> 4;
    auto xo = [&](int q) { return 16 * (q & 1) + xl; };
    auto yo = [&](int q, int r) { return 16 * (q >> 1) + 4 * r + yl; };
    auto inside = [&](int q, int r) { return xo(q) < L && yo(q, r) < L; };
    const int ax = a % L, ay = a / L, ex = e % L, ey = e / L;
    double* rows = filt + c.filt_off + (int64_t)p * L_tau * N;
    constexpr bool ck = CK;  // ckpt is given exactly for CK
    const int K = ck ? c.ck_k : 1;
    double* ckrows = ck ? ckpt + c.ck_row_off + (int64_t)p * c.ck_n * N : nullptr;
    double* seg = ck ? ckpt + g.seg_off + (int64_t)wv * (K - 1) * N : nullptr;
    auto ring_row = [&](int j) -> double* {
        if (!ck) return rows + (int64_t)j * N;
        const int sj = j / K, i = j - sj * K;
        return i == 0 ? ckrows + (int64_t)sj * N : seg + (int64_t)(i - 1) * N;
    };
    auto store_row = [&](double* row, const Tile64& F) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (inside(q, r)) row[yo(q, r) * L + xo(q)] = F.t[q][r];
    };
    // one step f~_j = W~_l . (C f~_{j-1} C) / total; returns the total
    auto step = [&](int l, Tile64& F) -> double {
        const double* Wl = Wsp + (int64_t)l * N;
        double w[16];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) w[4 * q + r] = Wl[inside(q, r) ? yo(q, r) * L + xo(q) : 0];
        __builtin_amdgcn_sched_barrier(0);  // W in flight during the matrix work
        const Tile64 H = circ64(circ64(F, Cb), Cb);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                F.t[q][r] = H.t[q][r] * w[4 * q + r];
                sum += F.t[q][r];
            }
        const double tot = wave_sum_f64(sum);
        if ((!(tot > 0.0) || !isfinite(tot)) && real && lane == 0)
            set_status(status, FH_ERR_NONFINITE, g.chain);
        const double inv = 1.0 / tot;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) F.t[q][r] *= inv;
        return tot;
    };
    // ---- forward pass over the ring, every row (every K-th with checkpoints) stored
    Tile64 F;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) F.t[q][r] = (xo(q) == ax && yo(q, r) == ay) ? 1.0 : 0.0;
    if (real) store_row(ring_row(0), F);
    double la = coef * aux[c.aux_off + (int64_t)anchor * N + a];
    for (int j = 1; j < L_tau; ++j) {
        const int l = (anchor + j) % L_tau;
        const double tot = step(l, F);
        la += log(tot) + shift[l];
        if (real && j % K == 0) store_row(ring_row(j), F);
    }
    {
        const Tile64 H = circ64(circ64(F, Cb), Cb);
        const int qe = 2 * (ey >> 4) + (ex >> 4), re = (ey & 15) >> 2;
        double hv = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (q == qe && r == re) hv = H.t[q][r];
        hv = __shfl(hv, (ex & 15) + 16 * (ey & 3), 64);
        if (real && lane == 0) {
            if (!(hv > 0.0)) set_status(status, FH_ERR_NONFINITE, g.chain);
            blk_logz[c.blk_off + (int64_t)p * c.nb] = la + log(hv);
        }
    }
    __syncthreads();  // every row of the group is stored before any wavefront reads one back
    // ---- backward messages
    Tile64 U;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) U.t[q][r] = (xo(q) == ex && yo(q, r) == ey) ? 1.0 : 0.0;
    double dt = 0.0;
    double* slab = gpart + g.part_off;
    for (int j = L_tau - 1; j >= 0; --j) {
        const int l = (anchor + j) % L_tau;
        if (ck && j % K != 0 && (j == L_tau - 1 || (j + 1) % K == 0)) {
            // entering segment j / K from above: its rows from the checkpoint (k_grad_mfma)
            const int j0 = j - j % K;
            const double* c0 = ring_row(j0);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double f0 = c0[inside(q, r) ? yo(q, r) * L + xo(q) : 0];
                    F.t[q][r] = inside(q, r) ? f0 : 0.0;
                }
            for (int i = j0 + 1; i <= j; ++i) {
                step((anchor + i) % L_tau, F);
                store_row(ring_row(i), F);
            }
        }
        // this slice's filter row and W: issued before the matrix work, waited for after it
        const double* row = ring_row(j);
        const double* Wl = Wsp + (int64_t)l * N;
        double fj[16], wl[16];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = inside(q, r) ? yo(q, r) * L + xo(q) : 0;
                fj[4 * q + r] = row[o];
                wl[4 * q + r] = Wl[o];
            }
        __builtin_amdgcn_sched_barrier(0);
        const Tile64 B = circ64(circ64(U, Cb), Cb);  // beta_j = C u_{j+1} C
        double den = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool in = inside(q, r);
                const int x = xo(q), y = yo(q, r);
                fj[4 * q + r] = in ? fj[4 * q + r] : 0.0;
                den += fj[4 * q + r] * B.t[q][r];
                const double bv = in ? B.t[q][r] : 0.0;
                // rows past L - 1 are not written: row L's slot holds the halo copy of row 0
                if (y < L) bt[wv][(y + 1) * 32 + x] = bv;
                if (y == L - 1) bt[wv][x] = bv;                 // halo row -1
                if (y == 0) bt[wv][(L + 1) * 32 + x] = bv;      // halo row L
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double num = 0.0;
        {
            const double* btw = bt[wv] + yl * 32;  // row lane / 16 - 1 of the halo layout
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int x = xo(q);
                const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = 16 * (q >> 1) + 4 * r;  // y = lane / 16 + rr
                    const double nbr = btw[(rr + 1) * 32 + xp] + btw[(rr + 1) * 32 + xm] +
                                       btw[(rr + 2) * 32 + x] + btw[rr * 32 + x];
                    num += inside(q, r) ? fj[4 * q + r] * nbr : 0.0;
                }
            }
        }
        const double dden = wave_sum_f64(den);
        const double dnum = wave_sum_f64(num);
        dt += dtau * dnum / dden;
        const double k = real ? coef / dden : 0.0;
        double* mgb = mg[j & 1][wv];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) mgb[yo(q, r) * 32 + xo(q)] = k * fj[4 * q + r] * B.t[q][r];
        __syncthreads();  // one barrier per slice: the tiles of slice j + 2 reuse these buffers
        {
            const double* m0 = mg[j & 1][0];
            const double* m1 = mg[j & 1][1];
            const double* m2 = mg[j & 1][2];
            const double* m3 = mg[j & 1][3];
            double* srow = slab + (int64_t)l * N;
            for (int i = threadIdx.x; i < 1024; i += kThreads) {
                const int yy = i >> 5, xx = i & 31;
                if (xx < L && yy < L) srow[yy * L + xx] = (m0[i] + m1[i]) + (m2[i] + m3[i]);
            }
        }
        if (j > 0) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool in = inside(q, r);
                    U.t[q][r] = in ? wl[4 * q + r] * B.t[q][r] : 0.0;
                    sum += U.t[q][r];
                }
            const double tot = wave_sum_f64(sum);
            if ((!(tot > 0.0) || !isfinite(tot)) && real && lane == 0)
                set_status(status, FH_ERR_NONFINITE, g.chain);
            const double inv = 1.0 / tot;
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) U.t[q][r] *= inv;
        }
    }
    if (real && lane == 0) dt_out[c.part_off + p] = dt;
}

// grad_aux[chain][l][r] = sum over the chain's groups, in group order, of the partial slabs.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gpart_reduce(const ChainInfo* __restrict__ chains,
                                                           int n_chains,
                                                           const GroupTask* __restrict__ groups,
                                                           const T* __restrict__ gpart,
                                                           T* __restrict__ grad,
                                                           int64_t aux_elems) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < aux_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_chains - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (chains[mid].aux_off <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const ChainInfo& c = chains[lo];
        // a chain's group slabs are consecutive, [L_tau][N] apart: eight loads in flight, the
        // sum still taken in group order
        const int64_t stride = (int64_t)c.L_tau * c.N;
        const T* src = gpart + groups[c.g0].part_off + (e - c.aux_off);
        const int n = c.g1 - c.g0;
        T s = T(0);
        int q = 0;
        for (; q + 8 <= n; q += 8) {
            T v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = src[(int64_t)(q + k) * stride];
#pragma unroll
            for (int k = 0; k < 8; ++k) s += v[k];
        }
        for (; q < n; ++q) s += src[(int64_t)q * stride];
        grad[e] = s;
    }
}

// The forward kernel classes of a split-bf16 plan whose chains take several of them (32 x 32
// pairs, padded tiles, packed 2 x 2 and 4 x 4 tiles) in one launch: workgroups [0, b1) run the
// pair kernel's tasks, [b1, b2) the padded tiles', [b2, b3) the 2 x 2 packed tiles', the rest
// the 4 x 4 ones', each class with the arithmetic of its own kernel. Once the chains cluster,
// each class is a few recursions of up to L_tau - 1 dependent steps; side by side, the pass
// takes the longest of them instead of their sum.
struct FwdClasses {
    const PairTask* pairs;
    const PairTask* cpairs;
    const int32_t* n_cpairs;
    const DrawTask* singles;
    const DrawTask* csingles;
    const int32_t* n_csingles;
    const PackTask* pack2;
    const PackTask* cpack2;
    const int32_t* n_cpack2;
    const PackTask* pack4;
    const PackTask* cpack4;
    const int32_t* n_cpack4;
    int32_t n_pairs, n_singles, n_pack2, n_pack4;
    int32_t b1, b2, b3;
};

__global__ __launch_bounds__(kThreads, 2) void k_forward_classes(
    const ChainInfo* __restrict__ chains, const uint16_t* __restrict__ cmat,
    const uint16_t* __restrict__ cmatp, const float* __restrict__ aux, const float* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, float* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const Rescue rsc, const NegPairs neg, double* __restrict__ blk_la,
    float* __restrict__ endrow, const int32_t* __restrict__ prep, const FwdClasses fc) {
    const int b = blockIdx.x, w = threadIdx.x >> 6;
    auto task = [&](int b0) { return __builtin_amdgcn_readfirstlane((b - b0) * kWaves + w); };
    if (b < fc.b1)
        forward_mfma2_body<32>(task(0), chains, fc.pairs, fc.n_pairs, cmat, aux, W, wshift,
                               aux_elems, total_slices, paths, perm, filt, blk_logz, sweep_ptr,
                               status, rsc, neg, blk_la, endrow, fc.cpairs, fc.n_cpairs);
    else if (b < fc.b2)
        forward_mfma_body<0>(task(fc.b1), chains, fc.singles, fc.n_singles, cmat, aux, W, wshift,
                             aux_elems, total_slices, paths, perm, filt, blk_logz, sweep_ptr,
                             status, rsc, neg, blk_la, endrow, fc.csingles, fc.n_csingles);
    else if (b < fc.b3)
        forward_pack_body<2, kPackTiles>(task(fc.b2), chains, fc.pack2, fc.n_pack2, cmatp, aux, W,
                                         wshift, aux_elems, total_slices, paths, perm, filt,
                                         blk_logz, sweep_ptr, status, rsc, neg, blk_la, endrow,
                                         fc.cpack2, fc.n_cpack2, prep);
    else
        forward_pack_body<4, kPackTiles>(task(fc.b3), chains, fc.pack4, fc.n_pack4, cmatp, aux, W,
                                         wshift, aux_elems, total_slices, paths, perm, filt,
                                         blk_logz, sweep_ptr, status, rsc, neg, blk_la, endrow,
                                         fc.cpack4, fc.n_cpack4, prep);
}

}  // namespace

hipError_t launch_forward_dmfma(fh_plan p, const void* aux, const int32_t* paths, hipStream_t s) {
    // fwdd_tasks: the L <= 32 tasks, then those of the 64 x 64 chains, then of the 48 x 48 ones
    const int32_t n2 = p->n_fwdd_tasks, n4 = p->n_fwdd4_tasks, n3 = p->n_fwdd3_tasks;
    auto blocks = [](int32_t n) { return (unsigned)((n + kWaves - 1) / kWaves); };
    if (n2 > 0)
        hipLaunchKernelGGL(k_forward_dmfma, dim3(blocks(n2)), dim3(kThreads), 0, s, p->d.chains,
                           p->d.fwdd_tasks, n2, p->d.cmat64, (const double*)aux,
                           (const double*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, p->d.perm, (double*)p->d.filt, p->d.blk_logz, p->d.sweep,
                           p->d.status);
    if (n4 > 0)
        hipLaunchKernelGGL(k_forward_dmfma_big<4>, dim3(blocks(n4)), dim3(kThreads), 0, s,
                           p->d.chains, p->d.fwdd_tasks + n2, n4, p->d.cmat64,
                           (const double*)aux, (const double*)p->d.W, p->d.wshift, p->aux_elems,
                           p->total_slices, paths, p->d.perm, (double*)p->d.filt, p->d.blk_logz,
                           p->d.sweep, p->d.status);
    if (n3 > 0)
        hipLaunchKernelGGL(k_forward_dmfma_big<3>, dim3(blocks(n3)), dim3(kThreads), 0, s,
                           p->d.chains, p->d.fwdd_tasks + n2 + n4, n3, p->d.cmat64,
                           (const double*)aux, (const double*)p->d.W, p->d.wshift, p->aux_elems,
                           p->total_slices, paths, p->d.perm, (double*)p->d.filt, p->d.blk_logz,
                           p->d.sweep, p->d.status);
    return hipGetLastError();
}

hipError_t launch_forward_mfma(fh_plan p, const void* aux, const int32_t* paths, hipStream_t s) {
    const bool shared_packs = p->d.fwdpc_tasks && !p->share_off;
    auto blocks_for = [](int32_t n) { return (int32_t)((n + kWaves - 1) / kWaves); };
    const int classes = (p->n_fwd32_tasks > 0) + (p->n_fwdx_tasks > 0) + (p->n_fwdp2_tasks > 0) +
                        (p->n_fwdp4_tasks > 0);
    if (classes > 1) {  // one launch for every class but the 64 x 64 sub-tiles
        FwdClasses fc;
        fc.pairs = p->d.fwd32_tasks;
        fc.cpairs = p->d.fwd32c_tasks;
        fc.n_cpairs = p->d.fwd32c_tasks && !p->share_off ? p->d.rescue + 5 : nullptr;
        fc.singles = p->d.fwdx_tasks;
        fc.csingles = p->d.fwdxc_tasks;
        fc.n_csingles = p->d.fwdxc_tasks && !p->share_off ? p->d.rescue + 7 : nullptr;
        fc.pack2 = p->d.fwdp_tasks;
        fc.cpack2 = p->d.fwdpc_tasks;
        fc.n_cpack2 = shared_packs ? p->d.rescue + 8 : nullptr;
        fc.pack4 = p->d.fwdp_tasks + p->n_fwdp2_tasks;
        fc.cpack4 = p->d.fwdpc_tasks ? p->d.fwdpc_tasks + p->n_fwdp2_tasks : nullptr;
        fc.n_cpack4 = shared_packs ? p->d.rescue + 9 : nullptr;
        fc.n_pairs = p->n_fwd32_tasks;
        fc.n_singles = p->n_fwdx_tasks;
        fc.n_pack2 = p->n_fwdp2_tasks;
        fc.n_pack4 = p->n_fwdp4_tasks;
        fc.b1 = blocks_for(p->n_fwd32_tasks);
        fc.b2 = fc.b1 + blocks_for(p->n_fwdx_tasks);
        fc.b3 = fc.b2 + blocks_for(p->n_fwdp2_tasks);
        const int32_t blocks = fc.b3 + blocks_for(p->n_fwdp4_tasks);
        hipLaunchKernelGGL(k_forward_classes, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           p->d.chains, p->d.cmat, p->d.cmatp, (const float*)aux,
                           (const float*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz, p->d.sweep,
                           p->d.status, rescue_args(p), kNegPairs, p->d.blk_la, p->d.endrow,
                           p->d.prep, fc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // L = 32 chains: worldline pairs per wavefront; other chains: one padded tile each
    if (classes == 1 && p->n_fwd32_tasks > 0) {
        const bool dense = p->d.fwd32c_tasks && !p->share_off;
        const unsigned blocks =
            (unsigned)((p->n_fwd32_tasks + kWaves - 1) / kWaves + (dense ? kXcds : 0));
        hipLaunchKernelGGL(k_forward_mfma2<32>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->d.fwd32_tasks, p->n_fwd32_tasks, p->d.cmat, (const float*)aux,
                           (const float*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz, p->d.sweep, p->d.status,
                           rescue_args(p), kNegPairs, p->d.blk_la, p->d.endrow,
                           p->d.fwd32c_tasks,
                           p->d.fwd32c_tasks && !p->share_off ? p->d.rescue + 5 : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (classes == 1 && p->n_fwdx_tasks > 0) {
        const unsigned blocks = (unsigned)((p->n_fwdx_tasks + kWaves - 1) / kWaves);
        hipLaunchKernelGGL(k_forward_mfma<0>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->d.fwdx_tasks, p->n_fwdx_tasks, p->d.cmat, (const float*)aux,
                           (const float*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz, p->d.sweep, p->d.status,
                           rescue_args(p), kNegPairs, p->d.blk_la, p->d.endrow, p->d.fwdxc_tasks,
                           p->d.fwdxc_tasks && !p->share_off ? p->d.rescue + 7 : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (p->n_fwd64_tasks > 0) {  // L = 64: four sub-tiles per worldline
        const unsigned blocks = (unsigned)((p->n_fwd64_tasks + kWaves - 1) / kWaves);
        hipLaunchKernelGGL(k_forward_mfma64<false>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->d.fwd64_tasks, p->n_fwd64_tasks, p->d.cmatb, (const float*)aux,
                           (const float*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz, p->d.sweep, p->d.status,
                           rescue_args(p), kNegPairs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // 32 < L < 64, padded to the 64 x 64 sub-tiles: after the L = 64 tasks in fwd64_tasks
    if (p->n_fwd64p_tasks > 0) {
        const unsigned blocks = (unsigned)((p->n_fwd64p_tasks + kWaves - 1) / kWaves);
        hipLaunchKernelGGL(k_forward_mfma64<true>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->d.fwd64_tasks + p->n_fwd64_tasks, p->n_fwd64p_tasks, p->d.cmatb,
                           (const float*)aux, (const float*)p->d.W, p->d.wshift, p->aux_elems,
                           p->total_slices, paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz,
                           p->d.sweep, p->d.status, rescue_args(p), kNegPairs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // small lattices, packed block-diagonally: L <= 16 two-by-two, L <= 8 four-by-four; with
    // shared filters, tiles of representatives from k_dedup's dense lists
    if (classes == 1 && p->n_fwdp2_tasks > 0) {
        const unsigned blocks = (unsigned)((p->n_fwdp2_tasks + kWaves - 1) / kWaves);
        hipLaunchKernelGGL((k_forward_pack<2, kPackTiles>), dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->d.fwdp_tasks, p->n_fwdp2_tasks, p->d.cmatp, (const float*)aux,
                           (const float*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz, p->d.sweep, p->d.status,
                           rescue_args(p), kNegPairs, p->d.blk_la, p->d.endrow, p->d.fwdpc_tasks,
                           shared_packs ? p->d.rescue + 8 : nullptr, p->d.prep);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (classes == 1 && p->n_fwdp4_tasks > 0) {
        const unsigned blocks = (unsigned)((p->n_fwdp4_tasks + kWaves - 1) / kWaves);
        hipLaunchKernelGGL((k_forward_pack<4, kPackTiles>), dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->d.fwdp_tasks + p->n_fwdp2_tasks, p->n_fwdp4_tasks, p->d.cmatp,
                           (const float*)aux, (const float*)p->d.W, p->d.wshift, p->aux_elems,
                           p->total_slices, paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz,
                           p->d.sweep, p->d.status, rescue_args(p), kNegPairs, p->d.blk_la,
                           p->d.endrow, p->d.fwdpc_tasks + p->n_fwdp2_tasks,
                           shared_packs ? p->d.rescue + 9 : nullptr, p->d.prep);
    }
    return hipGetLastError();
}

hipError_t launch_grad_mfma(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor,
                            void* grad_aux, hipStream_t s) {
    bool all32 = true;
    for (const ChainInfo& c : p->chains) all32 = all32 && c.L == 32;
    const bool ck = p->d.ckpt != nullptr;
    auto kern = all32 ? (ck ? k_grad_mfma<32, true> : k_grad_mfma<32, false>)
                      : (ck ? k_grad_mfma<0, true> : k_grad_mfma<0, false>);
    hipLaunchKernelGGL(kern, dim3(p->n_groups), dim3(kThreads), 0, s, p->d.chains,
                       p->d.group_tasks, p->d.cmat, (const float*)aux, (const float*)p->d.W,
                       p->d.wshift, p->aux_elems, p->total_slices, paths, (float*)p->d.filt,
                       (float*)p->d.gpart, p->d.blk_logz, p->d.dt, anchor, p->d.perm,
                       p->d.status, kNegPairs, (float*)p->d.ckpt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !grad_aux) return e;
    return launch_gpart_reduce(p, grad_aux, s);
}

hipError_t launch_gpart_reduce(fh_plan p, void* grad_aux, hipStream_t s) {
    int64_t b = (p->aux_elems + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    if (p->precision == FH_FP64)
        hipLaunchKernelGGL(k_gpart_reduce<double>, dim3((unsigned)b), dim3(kThreads), 0, s,
                           p->d.chains, p->n_chains, p->d.group_tasks, (const double*)p->d.gpart,
                           (double*)grad_aux, p->aux_elems);
    else
        hipLaunchKernelGGL(k_gpart_reduce<float>, dim3((unsigned)b), dim3(kThreads), 0, s,
                           p->d.chains, p->n_chains, p->d.group_tasks, (const float*)p->d.gpart,
                           (float*)grad_aux, p->aux_elems);
    return hipGetLastError();
}

hipError_t launch_grad_dmfma(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor,
                             void* grad_aux, hipStream_t s) {
    hipLaunchKernelGGL(p->d.ckpt ? k_grad_dmfma<true> : k_grad_dmfma<false>, dim3(p->n_groups),
                       dim3(kThreads), 0, s, p->d.chains,
                       p->d.group_tasks, p->d.cmat64, (const double*)aux, (const double*)p->d.W,
                       p->d.wshift, p->aux_elems, p->total_slices, paths, (double*)p->d.filt,
                       (double*)p->d.gpart, p->d.blk_logz, p->d.dt, anchor, p->d.perm,
                       p->d.status, (double*)p->d.ckpt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !grad_aux) return e;
    return launch_gpart_reduce(p, grad_aux, s);
}

}  // namespace fh
