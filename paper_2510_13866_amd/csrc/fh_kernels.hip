// gfx950 kernels of the FFBS worldline sweep: site potentials, FFT forward filter, backward
// inverse-CDF sampler, occupancy + Gibbs field draw, and the adjoint of the forward filter.
//
// Forward filter (Sec. 3.5.2, eq. ffbsFwd in the site basis): one workgroup advances two
// worldlines of the same (chain, spin) at once, packed as the real and imaginary parts of one
// complex L x L tile: the kinetic step G * f is IFFT(ghat . FFT(f)) with a real, even ghat, so
// it maps f_a + i f_b to (G * f_a) + i (G * f_b) exactly. The tile and a ping-pong buffer live
// in LDS; each radix-2/3/4 Stockham stage is one butterfly per thread between barriers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>
#include <math.h>

#include "fh_dmfma.h"
#include "fh_internal.h"
#include "fh_philox.h"

// Per-slice rows of fh_measure_noalloc (S(k) and C(r) of every slice, then the two site sums of
// every slice), held in this device array for callers that cannot allocate. Each GPU the library
// runs on holds one copy for the life of the process; its device address is taken once per
// device (fh::scratch_address) and passed to the kernels like any other buffer. Every element a
// call reads is written by the same call first, so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[fh::kScratchDoubles];

namespace fh {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ inline void set_status(int32_t* st, int code, int chain) {
    if (atomicCAS(&st[0], 0, code) == 0) atomicExch(&st[1], chain);
}

// Largest c with key(c) <= v over chains sorted by that key.
template <typename F>
__device__ inline int find_chain(int n, int64_t v, F key) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key(mid) <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum of K doubles (same order every call). red: LDS, K*kWaves doubles.
template <int K>
__device__ inline void block_sum(double (&v)[K], double* red) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) red[i * kWaves + w] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += red[i * kWaves + q];
        v[i] = s;
    }
    __syncthreads();
}

// 2D FFT of the L x L tile in A (S is scratch). Callers synchronise before the call; the
// result is back in A because both dimensions take the same (even total) number of stages.
template <typename T, bool INV>
__device__ inline void fft2d(cpx<T>* A, cpx<T>* S, int L, const RadixPlan& rp,
                             const cpx<T>* tw) {
    cpx<T>* src = A;
    cpx<T>* dst = S;
    for (int dim = 0; dim < 2; ++dim) {
        const int ls = dim == 0 ? L : 1, es = dim == 0 ? 1 : L;
        int Ns = 1;
        for (int st = 0; st < rp.n; ++st) {
            const int p = rp.rad[st];
            const int nbf = L * (L / p);
            for (int b = threadIdx.x; b < nbf; b += blockDim.x)
                stockham_butterfly_rt<T, INV>(p, b, L, Ns, ls, es, src, dst, tw);
            __syncthreads();
            Ns *= p;
            cpx<T>* t = src;
            src = dst;
            dst = t;
        }
    }
}

template <typename T>
struct FftLds {
    cpx<T>* A;
    cpx<T>* S;
    cpx<T>* U;
    cpx<T>* tw;
    double* g;
    double* red;
};

template <typename T>
__device__ inline FftLds<T> carve(unsigned char* smem, int maxN, int maxL, bool third) {
    FftLds<T> l;
    size_t off = 0;
    l.A = (cpx<T>*)(smem + off);
    off += sizeof(cpx<T>) * maxN;
    l.S = (cpx<T>*)(smem + off);
    off += sizeof(cpx<T>) * maxN;
    l.U = third ? (cpx<T>*)(smem + off) : nullptr;
    if (third) off += sizeof(cpx<T>) * maxN;
    l.tw = (cpx<T>*)(smem + off);
    off += sizeof(cpx<T>) * maxL;
    off = (off + 7) & ~(size_t)7;
    l.g = (double*)(smem + off);
    off += sizeof(double) * maxL;
    l.red = (double*)(smem + off);
    return l;
}

template <typename T>
__device__ inline void load_chain_tables(const ChainInfo& c, const double* tables, FftLds<T>& l) {
    const double* tw = tables + tab_tw(c);
    const double* g = tables + tab_g(c);
    for (int m = threadIdx.x; m < c.L; m += blockDim.x) {
        l.tw[m] = {(T)tw[2 * m], (T)tw[2 * m + 1]};
        l.g[m] = g[m];
    }
}

__device__ inline int checked_site(int r, int N, int32_t* status, int chain) {
    if (r < 0 || r >= N) {
        set_status(status, FH_ERR_BAD_PATH, chain);
        return 0;
    }
    return r;
}

// Forward recursion of one block for a pair of worldlines (Sec. 3.5.2):
//   f~_0 = delta_a; h_j = W~_{start+j} . (G * f~_{j-1}); c_j = sum h_j; f~_j = h_j / c_j
//   log Z = coef aux_start(a) + sum_j (log c_j + m_{start+j}) + log (G * f~_{len-1})(e),
// with W~ = W exp(-m) the shifted potentials, shift[l] = m_spin(l) and log W = coef * aux.
// Rows f~_j are stored at row + (j - jshift)*N for j >= 1 (and j = 0 when jshift == 0).
// The last step's end weight is a direct FP64 sum with the real-space kernel g(dx) g(dy).
// With `low` given (the FP32 sweep), a worldline whose step total or end weight falls below
// kRangeFloor is reported there (low[0], low[1]) for the FP64 re-filter instead of the status.
template <typename T>
__device__ void forward_pass(const ChainInfo& c, const double* tables, const T* Wsp,
                             const double* shift, const T* auxc, double coef, int start, int len,
                             int a_a, int e_a, int a_b,
                             int e_b, bool has_b, T* row_a, T* row_b, int jshift, FftLds<T>& l,
                             double* logz_a, double* logz_b, int32_t* status, int chain,
                             bool* low = nullptr) {
    // the sweep's FP32 rows hold f~ 2^row_exp; the adjoint's ring (jshift = 0) is unscaled
    const int rexp = jshift == 0 ? 0 : c.row_exp;
    const T sc = (T)ldexp(1.0, rexp);
    const double lsc = rexp * 0.69314718055994530942;
    const double floor = low ? (double)c.step_floor : 0.0;
    const double efloor = low ? kRangeFloorD : 0.0;
    bool low_a = false, low_b = false;
    const int N = c.N, L = c.L, L_tau = c.L_tau;
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        cpx<T> v = {r == a_a ? sc : T(0), (has_b && r == a_b) ? sc : T(0)};
        l.A[r] = v;
        if (jshift == 0) {
            row_a[r] = v.re;
            if (has_b) row_b[r] = v.im;
        }
    }
    // log W_start(a) straight from the field: exact, and immune to underflow of W~(a)
    double la = coef * (double)auxc[(int64_t)start * N + a_a] - lsc;
    double lb = has_b ? coef * (double)auxc[(int64_t)start * N + a_b] - lsc : 0.0;
    const double* gh = tables + tab_ghat(c);
    __syncthreads();
    for (int j = 1; j < len; ++j) {
        fft2d<T, false>(l.A, l.S, L, c.plan, l.tw);
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            const T m = (T)gh[k];
            l.A[k].re *= m;
            l.A[k].im *= m;
        }
        __syncthreads();
        fft2d<T, true>(l.A, l.S, L, c.plan, l.tw);
        const T* Wl = Wsp + (int64_t)((start + j) % L_tau) * N;
        double s[2] = {0.0, 0.0};
        for (int r = threadIdx.x; r < N; r += blockDim.x) {
            const T w = Wl[r];
            cpx<T> h = {l.A[r].re * w, l.A[r].im * w};
            l.A[r] = h;
            s[0] += (double)h.re;
            s[1] += (double)h.im;
        }
        block_sum<2>(s, l.red);
        const bool ba = !(s[0] > floor) || !isfinite(s[0]);
        const bool bb = has_b && (!(s[1] > floor) || !isfinite(s[1]));
        low_a = low_a || ba;
        low_b = low_b || bb;
        if (!low && (ba || bb) && threadIdx.x == 0) set_status(status, FH_ERR_NONFINITE, chain);
        const T ia = (T)((double)sc / s[0]);
        const T ib = has_b ? (T)((double)sc / s[1]) : T(0);
        const double m = shift[(start + j) % L_tau] - lsc;
        la += log(s[0]) + m;
        if (has_b) lb += log(s[1]) + m;
        T* ra = row_a + (int64_t)(j - jshift) * N;
        T* rb = has_b ? row_b + (int64_t)(j - jshift) * N : nullptr;
        for (int r = threadIdx.x; r < N; r += blockDim.x) {
            cpx<T> v = {l.A[r].re * ia, l.A[r].im * ib};
            l.A[r] = v;
            ra[r] = v.re;
            if (has_b) rb[r] = v.im;
        }
        __syncthreads();
    }
    const int eax = e_a % L, eay = e_a / L, ebx = e_b % L, eby = e_b / L;
    double z[2] = {0.0, 0.0};
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        const int x = r % L, y = r / L;
        int dx = eax - x, dy = eay - y;
        dx += dx < 0 ? L : 0;
        dy += dy < 0 ? L : 0;
        z[0] += l.g[dx] * l.g[dy] * (double)l.A[r].re;
        if (has_b) {
            dx = ebx - x;
            dy = eby - y;
            dx += dx < 0 ? L : 0;
            dy += dy < 0 ? L : 0;
            z[1] += l.g[dx] * l.g[dy] * (double)l.A[r].im;
        }
    }
    block_sum<2>(z, l.red);
    // an end site deeper in the filter's tail than the FFT resolves (~eps * max) can leave a
    // non-positive end weight: report it instead of returning log of it
    low_a = low_a || !(z[0] > efloor);
    low_b = low_b || (has_b && !(z[1] > efloor));
    if (low) {
        low[0] = low_a;
        low[1] = low_b;
    } else if ((low_a || low_b) && threadIdx.x == 0) {
        set_status(status, FH_ERR_NONFINITE, chain);
    }
    *logz_a = la + log(z[0]);
    *logz_b = has_b ? lb + log(z[1]) : 0.0;
}

// ---- kernels ----------------------------------------------------------------------------------

__global__ void k_set_u64(uint64_t* p, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_bump_u64(uint64_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = *p + 1;
}

__global__ void k_zero(uint32_t* p, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Site potentials of one (chain, slice) in log-domain-shifted form (eq. hirsch / eq. gaussHS):
// log W_spin(l, r) = coef_spin * aux(l, r); the tables hold W~ = exp(log W - m_spin(l)) with
// m_spin(l) = max_r log W_spin(l, r), so W~ <= 1 whatever the field (FP32 tables: m lowered by
// kWScaleLog2 ln 2, so W~ <= 2^60), and m is kept in FP64 and added back to log Z. Filters are
// normalised per step, so the shift changes nothing else.
// W[0 .. aux_elems) holds spin up, W[aux_elems .. 2 aux_elems) spin down.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_potentials(const ChainInfo* __restrict__ chains,
                                                         int n_chains, const T* __restrict__ aux,
                                                         T* __restrict__ W, double* __restrict__ wshift,
                                                         int64_t aux_elems, int64_t total_slices,
                                                         int32_t* status) {
    __shared__ double red[2 * kWaves];
    const int gs = blockIdx.x;
    const int ci = find_chain(n_chains, gs, [&](int i) { return chains[i].slice_off; });
    const ChainInfo& c = chains[ci];
    const int64_t base = c.aux_off + (int64_t)(gs - c.slice_off) * c.N;
    double mu = -INFINITY, md = -INFINITY;
    bool bad = false;
    for (int r = threadIdx.x; r < c.N; r += blockDim.x) {
        const double v = (double)aux[base + r];
        bad |= !isfinite(v);
        mu = fmax(mu, c.coef_up * v);
        md = fmax(md, c.coef_dn * v);
    }
    if (bad) set_status(status, FH_ERR_NONFINITE, ci);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mu = fmax(mu, __shfl_xor(mu, o, 64));
        md = fmax(md, __shfl_xor(md, o, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = mu;
        red[kWaves + w] = md;
    }
    __syncthreads();
    mu = red[0];
    md = red[kWaves];
    for (int q = 1; q < kWaves; ++q) {
        mu = fmax(mu, red[q]);
        md = fmax(md, red[kWaves + q]);
    }
    if (!isfinite(mu)) mu = 0.0;
    if (!isfinite(md)) md = 0.0;
    if (sizeof(T) == 4) {  // FP32 tables: W~ 2^kWScaleLog2, so W~ down to 2^-226 stays normal
        mu -= kWScaleLog2 * 0.69314718055994530942;
        md -= kWScaleLog2 * 0.69314718055994530942;
    }
    for (int r = threadIdx.x; r < c.N; r += blockDim.x) {
        const double v = (double)aux[base + r];
        W[base + r] = (T)exp(c.coef_up * v - mu);
        W[aux_elems + base + r] = (T)exp(c.coef_dn * v - md);
    }
    if (threadIdx.x == 0) {
        wshift[gs] = mu;
        wshift[total_slices + gs] = md;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_forward_fft(
    const ChainInfo* __restrict__ chains, const PairTask* __restrict__ tasks,
    const double* __restrict__ tables, const T* __restrict__ aux, const T* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm, T* __restrict__ filt,
    double* __restrict__ blk_logz, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    int maxN, int maxL, const Rescue rsc) {
    extern __shared__ __align__(16) unsigned char smem[];
    FftLds<T> l = carve<T>(smem, maxN, maxL, false);
    const PairTask t = tasks[blockIdx.x];
    const ChainInfo& c = chains[t.chain];
    // re-filtered whole in FP64 this pass (the whole workgroup leaves: no barrier is skipped)
    if (fp64_circulant(c.L) && rescue_held(rsc, t.chain)) return;
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const bool has_b = t.p_b >= 0;
    const int spin = t.p_a >= c.n_up ? 1 : 0;
    const T* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const int end = (start + len) % c.L_tau;
    const int32_t* pc = paths + c.path_off;
    // a block that runs past slice L_tau - 1 ends on the worldline its owner reconnects to
    const bool wraps = start + len >= c.L_tau;
    const int qa = wraps ? perm[c.part_off + t.p_a] : t.p_a;
    const int qb = has_b ? (wraps ? perm[c.part_off + t.p_b] : t.p_b) : 0;
    const int a_a = checked_site(pc[(int64_t)start * c.np + t.p_a], c.N, status, t.chain);
    const int e_a = checked_site(pc[(int64_t)end * c.np + qa], c.N, status, t.chain);
    const int a_b = has_b ? checked_site(pc[(int64_t)start * c.np + t.p_b], c.N, status, t.chain) : 0;
    const int e_b = has_b ? checked_site(pc[(int64_t)end * c.np + qb], c.N, status, t.chain) : 0;
    load_chain_tables(c, tables, l);
    const int64_t rowbase = (int64_t)t.block * (c.B - 1);
    T* row_a = filt + c.filt_off + ((int64_t)t.p_a * c.L_tau + rowbase) * c.N;
    T* row_b = has_b ? filt + c.filt_off + ((int64_t)t.p_b * c.L_tau + rowbase) * c.N : nullptr;
    double lza, lzb;
    bool low[2] = {false, false};  // FP32: the worldlines that left FP32's range
    forward_pass<T>(c, tables, Wsp, shift, aux + c.aux_off, spin ? c.coef_dn : c.coef_up, start,
                    len, a_a, e_a, a_b, e_b, has_b, row_a, row_b, 1, l, &lza, &lzb, status,
                    t.chain, rsc.words ? low : nullptr);
    if (threadIdx.x == 0) {
        blk_logz[c.blk_off + (int64_t)t.p_a * c.nb + t.block] = lza;
        if (has_b) blk_logz[c.blk_off + (int64_t)t.p_b * c.nb + t.block] = lzb;
        if (low[0]) rescue_push(rsc, c, t.chain, t.p_a, t.block, kCauseFft);
        if (has_b && low[1]) rescue_push(rsc, c, t.chain, t.p_b, t.block, kCauseFft);
    }
}

// logZ[particle] = sum over its blocks, in block order.
__global__ void k_logz_reduce(const ChainInfo* __restrict__ chains, int n_chains,
                              const double* __restrict__ blk_logz, double* __restrict__ logZ,
                              int64_t particles) {
    const int64_t gp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gp >= particles) return;
    const int c = find_chain(n_chains, gp, [&](int i) { return chains[i].part_off; });
    const ChainInfo& ci = chains[c];
    const int64_t p = gp - ci.part_off;
    double s = 0.0;
    for (int b = 0; b < ci.nb; ++b) s += blk_logz[ci.blk_off + p * ci.nb + b];
    logZ[gp] = s;
}

// A windowed chain's backward tasks sit in the windowed kernel's list and in a full-row
// kernel's list; the windowed kernel draws them unless k_bw_adapt has moved the plan to the
// full-row kernels for this pass (bw_state[0] > 0).
__device__ inline bool on_window(const ChainInfo* chains, int chain, const int32_t* bw_state) {
    return chains[chain].win_on && bw_state[0] == 0;
}

// Backward sampling, one wavefront per (chain, particle, block). For j = len-1 .. 1:
// w(r) = max(f~_j(r), 0) g(x_{j+1} - x) g(y_{j+1} - y) in FP64; lane l owns the contiguous sites
// [l E, (l+1) E); C_r = (exclusive scan of lane totals) + (running sum within the lane);
// the draw is the smallest r with C_r > u * C_total (Philox uniform), else the last r with w > 0.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_backward(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const double* __restrict__ tables, const T* __restrict__ filt, int32_t* __restrict__ paths,
    const int32_t* __restrict__ perm, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    const int32_t* __restrict__ bw_state, const Rescue rsc) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int task = blockIdx.x * kWaves + wv;
    if (task >= n_tasks) return;  // whole wavefront leaves; no block-level barrier below
    if (on_window(chains, tasks[task].chain, bw_state)) return;  // k_backward_win draws it
    const DrawTask t = tasks[task];
    const ChainInfo& c = chains[t.chain];
    if (rescue_queued(rsc, c, t.p, t.block)) return;  // k_rescue redraws it in FP64
    const uint64_t sweep = *sweep_ptr;
    int start, len;
    block_of(c, sweep, t.block, &start, &len);
    if (len < 2) return;
    const int N = c.N, L = c.L;
    const double* __restrict__ g = tables + tab_g(c);
    int32_t* pc = paths + c.path_off;
    const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
    int cur = checked_site(pc[(int64_t)((start + len) % c.L_tau) * c.np +
                              (start + len >= c.L_tau ? qn : t.p)], N, status, t.chain);
    const int E = (N + 63) / 64;
    const int i0 = lane * E;
    const int i1 = min(i0 + E, N);
    const int ro = row_owner(rsc, c, t.p, t.block);  // shared forward filters
    const T* rows = filt + c.filt_off + ((int64_t)ro * c.L_tau + (int64_t)t.block * (c.B - 1)) * N;
    for (int j = len - 1; j >= 1; --j) {
        const int l = (start + j) % c.L_tau;
        const T* f = rows + (int64_t)(j - 1) * N;
        const int cx = cur % L, cy = cur / L;
        double tot = 0.0;
        for (int i = i0; i < i1; ++i) {
            const int x = i % L, y = i / L;
            int dx = cx - x, dy = cy - y;
            dx += dx < 0 ? L : 0;
            dy += dy < 0 ? L : 0;
            const double fv = (double)f[i];
            tot += (fv > 0.0 ? fv : 0.0) * g[dx] * g[dy];
        }
        double incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double up = __shfl_up(incl, o, 64);
            if (lane >= o) incl += up;
        }
        double excl = __shfl_up(incl, 1, 64);
        if (lane == 0) excl = 0.0;
        const double total = __shfl(incl, 63, 64);
        int chosen = cur;
        if (rsc.words && (!(total > 0.0) || !isfinite(total))) {
            // no usable FP32 weight: the block is redrawn from FP64 filters
            if (lane == 0) rescue_push(rsc, c, t.chain, t.p, t.block, kCauseDraw);
            return;
        }
        if (!(total > 0.0) || !isfinite(total)) {
            if (lane == 0)
                set_status(status, isfinite(total) ? FH_ERR_ZERO_WEIGHT : FH_ERR_NONFINITE, t.chain);
        } else {
            const u64x4 rnd = philox4x64_10((uint64_t)t.p, (uint64_t)l, sweep, kTagPath, c.seed, 0);
            const double T_ = u01_from(rnd.x0) * total;
            double run = excl;
            int first = 0x7fffffff, lastpos = -1;
            for (int i = i0; i < i1; ++i) {
                const int x = i % L, y = i / L;
                int dx = cx - x, dy = cy - y;
                dx += dx < 0 ? L : 0;
                dy += dy < 0 ? L : 0;
                const double fv = (double)f[i];
                const double w = (fv > 0.0 ? fv : 0.0) * g[dx] * g[dy];
                run += w;
                if (first == 0x7fffffff && run > T_) first = i;
                if (w > 0.0) lastpos = i;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                first = min(first, __shfl_xor(first, o, 64));
                lastpos = max(lastpos, __shfl_xor(lastpos, o, 64));
            }
            chosen = first != 0x7fffffff ? first : lastpos;
            if (chosen < 0) chosen = cur;
            // FP32 plans: a site drawn from a filter value near FP32's floor (kRangeFloor)
            if (rsc.words && !((double)f[chosen] >= kRangeFloorD)) {
                if (lane == 0) rescue_push(rsc, c, t.chain, t.p, t.block, kCauseDraw);
                return;
            }
        }
        if (lane == 0) pc[(int64_t)l * c.np + (start + j >= c.L_tau ? qn : t.p)] = chosen;
        cur = chosen;
    }
}

// Cross-lane helpers on DPP and readlane (no LDS crossbar).
template <int CTRL>
__device__ inline double dpp_f64(double v) {  // value of the DPP source lane, 0 where none
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    // bound_ctrl: a lane without a source lane reads 0, so no zeroed destination is needed
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}
__device__ inline double readlane_f64(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}
// Inclusive prefix sum over the 64 lanes (Hillis-Steele inside each row of 16 lanes with
// row_shr, then the three preceding row totals); *total receives the sum of all lanes.
__device__ inline double wave_incl_scan_f64(double v, int lane, double* total) {
    v += dpp_f64<0x111>(v);  // row_shr:1
    v += dpp_f64<0x112>(v);  // row_shr:2
    v += dpp_f64<0x114>(v);  // row_shr:4
    v += dpp_f64<0x118>(v);  // row_shr:8
    const double r0 = readlane_f64(v, 15), r1 = readlane_f64(v, 31), r2 = readlane_f64(v, 47);
    const double r3 = readlane_f64(v, 63);
    const int row = lane >> 4;
    const double base = row == 0 ? 0.0 : row == 1 ? r0 : row == 2 ? r0 + r1 : (r0 + r1) + r2;
    *total = ((r0 + r1) + r2) + r3;
    return v + base;
}

// Backward sampling for N <= 1024, same draw rule as k_backward: the lane's weights stay in
// registers between the scan and the search, filter rows are prefetched ahead (two rows in FP32,
// one in FP64; 16-byte loads for 32 x 32 lattices), g lives in LDS, and lane k computes the
// Philox uniform of draw s = 64 b + k once per 64 draws. E = sites per lane this body handles;
// LFIX = 32 is the branch-free full-tile case.
template <typename T, bool VEC, int LFIX, int E>
__device__ void backward_task(const DrawTask& t, const ChainInfo& c, const double* g,
                              const T* __restrict__ filt, int32_t* __restrict__ paths,
                              const int32_t* __restrict__ perm, uint64_t sweep, int32_t* status,
                              int lane, const Rescue rsc, const T* rows_at = nullptr) {
    constexpr int DEPTH = sizeof(T) == 4 ? 2 : 1;  // rows in flight ahead of the current one
    int start, len;
    block_of(c, sweep, t.block, &start, &len);
    if (len < 2) return;
    if (rescue_queued(rsc, c, t.p, t.block)) return;  // k_rescue redraws it in FP64
    const int L = LFIX ? LFIX : c.L, N = LFIX ? LFIX * LFIX : c.N, L_tau = c.L_tau;
    int32_t* pc = paths + c.path_off;
    const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
    int cur = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                              (start + len >= L_tau ? qn : t.p)], N, status, t.chain);
    const int per = LFIX ? (LFIX * LFIX) / 64 : (N + 63) / 64;  // sites per lane (<= E)
    const int i0 = lane * per;
    const int cnt = LFIX ? per : max(0, min(per, N - i0));
    const int x0 = cnt > 0 ? i0 % L : 0, y0 = cnt > 0 ? i0 / L : 0;
    // the block's rows in the plan's workspace, or at rows_at (the FP64 re-filter's slot)
    const T* rows = rows_at ? rows_at
                            : filt + c.filt_off + ((int64_t)row_owner(rsc, c, t.p, t.block) * L_tau +
                                                   (int64_t)t.block * (c.B - 1)) * N;
    // row of draw j is rows + (j - 1) N; draws run j = len-1 .. 1
    auto load_row = [&](int j, T (&dst)[E]) {
        const T* r = rows + (int64_t)(j - 1) * N + i0;
        if (VEC) {
            typedef T vec4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int q = 0; q < E / 4; ++q) {
                const vec4 v4 = *(const vec4*)(r + 4 * q);
                dst[4 * q] = v4[0];
                dst[4 * q + 1] = v4[1];
                dst[4 * q + 2] = v4[2];
                dst[4 * q + 3] = v4[3];
            }
        } else {
#pragma unroll
            for (int k = 0; k < E; ++k) dst[k] = k < cnt ? r[k] : T(0);
        }
    };
    T ring[DEPTH + 1][E];
#pragma unroll
    for (int d = 0; d <= DEPTH; ++d)
        if (len - 1 - d >= 1) load_row(len - 1 - d, ring[d]);
    double ureg = 0.0;
    for (int s = 0; s < len - 1; ++s) {
        const int j = len - 1 - s;
        if ((s & 63) == 0) {
            const int jj = j - lane;
            ureg = 0.0;
            if (jj >= 1) {
                const u64x4 r = philox4x64_10((uint64_t)t.p, (uint64_t)((start + jj) % L_tau),
                                              sweep, kTagPath, c.seed, 0);
                ureg = u01_from(r.x0);
            }
        }
        const double u = readlane_f64(ureg, s & 63);
        T f[E];
#pragma unroll
        for (int k = 0; k < E; ++k) f[k] = ring[0][k];
#pragma unroll
        for (int d = 0; d < DEPTH; ++d)
#pragma unroll
            for (int k = 0; k < E; ++k) ring[d][k] = ring[d + 1][k];
        if (j - 1 - DEPTH >= 1) load_row(j - 1 - DEPTH, ring[DEPTH]);
        const int cx = cur % L, cy = cur / L;
        double w[E];
        double tot = 0.0;
        if (LFIX == 32) {
            // 16 sites per lane, all in row y0: no wraps, no guards
            const double gy = g[(cy - y0) & 31];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const double fk = (double)f[k];
                const double wk = (fk > 0.0 ? fk : 0.0) * (gy * g[(cx - x0 - k) & 31]);
                w[k] = wk;
                tot += wk;
            }
        } else {
            int x = x0, y = y0;
            int dy = cy - y;
            dy += dy < 0 ? L : 0;
            double gy = g[dy];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                double wk = 0.0;
                if (k < cnt) {
                    int dx = cx - x;
                    dx += dx < 0 ? L : 0;
                    const double fk = (double)f[k];
                    wk = (fk > 0.0 ? fk : 0.0) * (gy * g[dx]);
                    if (++x == L) {
                        x = 0;
                        ++y;
                        dy = cy - y;
                        dy += dy < 0 ? L : 0;
                        gy = g[dy];
                    }
                }
                w[k] = wk;
                tot += wk;
            }
        }
        double total;
        const double incl = wave_incl_scan_f64(tot, lane, &total);
        double run = incl - tot;
        int chosen = cur;
        if (rsc.words && (!(total > 0.0) || !isfinite(total))) {
            // no usable FP32 weight: the block is redrawn from FP64 filters
            if (lane == 0) rescue_push(rsc, c, t.chain, t.p, t.block, kCauseDraw);
            return;
        }
        if (!(total > 0.0) || !isfinite(total)) {
            if (lane == 0)
                set_status(status, isfinite(total) ? FH_ERR_ZERO_WEIGHT : FH_ERR_NONFINITE, t.chain);
        } else {
            const double T_ = u * total;
            int first = -1;
            double fsel = 0.0;  // the filter value of the drawn site
#pragma unroll
            for (int k = 0; k < E; ++k) {
                run += w[k];
                if (first < 0 && k < cnt && run > T_) {
                    first = i0 + k;
                    fsel = (double)f[k];
                }
            }
            const uint64_t found = __ballot(first >= 0);
            if (found) {
                const int src = __ffsll((unsigned long long)found) - 1;
                chosen = __builtin_amdgcn_readlane(first, src);
                fsel = readlane_f64(fsel, src);
            } else {
                int lastpos = -1;
#pragma unroll
                for (int k = 0; k < E; ++k)
                    if (k < cnt && w[k] > 0.0) {
                        lastpos = i0 + k;
                        fsel = (double)f[k];
                    }
                const uint64_t has = __ballot(lastpos >= 0);
                if (has) {
                    const int src = 63 - __clzll((long long)has);
                    chosen = __builtin_amdgcn_readlane(lastpos, src);
                    fsel = readlane_f64(fsel, src);
                }
            }
            // FP32 plans: a site drawn from a filter value near FP32's floor (kRangeFloor)
            if (rsc.words && !(fsel >= kRangeFloorD)) {
                if (lane == 0) rescue_push(rsc, c, t.chain, t.p, t.block, kCauseDraw);
                return;
            }
        }
        if (lane == 0)
            pc[(int64_t)((start + j) % L_tau) * c.np + (start + j >= L_tau ? qn : t.p)] = chosen;
        cur = chosen;
    }
}

// Backward sampling for 32 x 32 lattices, one wavefront per (chain, worldline, block). Lane k
// owns the sites 16k .. 16k+15, all in lattice row y0 = k / 2 from column x0 = 16 (k % 2), read
// as four 16-byte loads per filter row. Given the next slice's site (cx, cy) the weight of site
// (x0 + i, y0) is max(f_i, 0) g(cx - x0 - i) g(cy - y0) (periodic differences). The lane keeps
// the FP64 prefix P_i = sum over i' <= i of max(f_i', 0) g(cx - x0 - i'); its total is
// g(cy - y0) P_15, and the wavefront scan of the totals gives run, the sum before the lane. The
// draw is the first site where run + g(cy - y0) P_i exceeds u times the grand total, tested as
// P_i > (u total - run) / g(cy - y0): the same comparison up to FP64 rounding. The lowest lane
// holding such a site supplies it. If rounding leaves none, the last site with a positive
// weight increment is taken, as the draw rule prescribes for that case.
//
// Rows are prefetched DEPTH draws ahead into DEPTH + 1 buffers, and the draw loop is unrolled by
// DEPTH + 1 so that no buffer moves between registers (a move would wait for the newest loads).
// Every load and store is unconditional, which lets each wait leave younger memory operations in
// flight: draws past the end of the block, padding the count to a multiple of DEPTH + 1, re-read
// row 1 and rewrite the value the last real draw stored. All lanes store the (uniform) draw.
template <typename T>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 ? 4 : 3) void k_backward_l32(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const double* __restrict__ tables, const T* __restrict__ filt, int32_t* __restrict__ paths, const int32_t* __restrict__ perm,
    const uint64_t* __restrict__ sweep_ptr, int32_t* status, const int32_t* __restrict__ bw_state,
    const Rescue rsc) {
    constexpr int DEPTH = sizeof(T) == 4 ? 2 : 1;
    constexpr int NB = DEPTH + 1;
    __shared__ double g2sh[kWaves][64];  // g2[m] = g(m mod 32), so g(d) = g2[d + 32] for |d| < 32
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int task = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wv);
    bool active = task < n_tasks && !on_window(chains, tasks[task].chain, bw_state);
    DrawTask t = {0, 0, 0, 0};
    if (active) {
        t = tasks[task];
        g2sh[wv][lane] = tables[tab_g(chains[t.chain]) + (lane & 31)];
        active = !rescue_queued(rsc, chains[t.chain], t.p, t.block);  // k_rescue draws it
    }
    __syncthreads();  // the only barrier; every wave reaches it
    if (!active) return;
    const ChainInfo& c = chains[t.chain];
    const uint64_t sweep = *sweep_ptr;
    int start, len;
    block_of(c, sweep, t.block, &start, &len);
    const int nd = len - 1;  // draw s sets slice start + (nd - s), s = 0 .. nd - 1
    if (nd < 1) return;
    const int L_tau = c.L_tau;
    int32_t* pc = paths + c.path_off;
    const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
    int cur = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                              (start + len >= L_tau ? qn : t.p)], 1024, status, t.chain);
    const int x0 = 16 * (lane & 1), y0 = lane >> 1;
    const int ro = row_owner(rsc, c, t.p, t.block);  // shared forward filters
    const T* rows = filt + c.filt_off + ((int64_t)ro * L_tau + (int64_t)t.block * (c.B - 1)) * 1024 +
                    16 * lane;
    typedef T vec4 __attribute__((ext_vector_type(4)));
    auto load_row = [&](int j, T (&dst)[16]) {  // row of draw slice start + j, j clamped to >= 1
        const T* r = rows + (int64_t)((j < 1 ? 1 : j) - 1) * 1024;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const vec4 v4 = *(const vec4*)(r + 4 * q);
            dst[4 * q] = v4[0];
            dst[4 * q + 1] = v4[1];
            dst[4 * q + 2] = v4[2];
            dst[4 * q + 3] = v4[3];
        }
    };
    T ring[NB][16];
#pragma unroll
    for (int b = 0; b < NB; ++b) {  // in draw order: the loop's first wait then spares the rest
        load_row(nd - b, ring[b]);
        __builtin_amdgcn_sched_barrier(0);
    }
    const double* g2 = g2sh[wv];
    double ureg = 0.0;
    int err = 0;  // the first error of the block, reported once after the loop (no atomics inside)
    const int nd_pad = (nd + NB - 1) / NB * NB;
    bool halted = false;  // the block left FP32's range: k_rescue redraws it
    for (int s0 = 0; s0 < nd_pad && !halted; s0 += NB) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int s = s0 + b;
            const bool real = s < nd && !halted;
            const int j = real ? nd - s : 1;
            if ((s & 63) == 0) {  // lane k draws the uniform of draw s + k
                const int jj = nd - s - lane;
                ureg = 0.0;
                if (jj >= 1) {
                    const u64x4 r = philox4x64_10((uint64_t)t.p, (uint64_t)((start + jj) % L_tau),
                                                  sweep, kTagPath, c.seed, 0);
                    ureg = u01_from(r.x0);
                }
            }
            const double u = readlane_f64(ureg, s & 63);
            const int cx = cur & 31, cy = cur >> 5;
            const double* gx = g2 + (cx - x0 + 17);  // g(cx - x0 - i) = gx[15 - i], index 1 .. 63
            const double gy = g2[cy - y0 + 32];
            double P[16];
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const double fi = (double)ring[b][i];
                acc = fma(fi > 0.0 ? fi : 0.0, gx[15 - i], acc);
                P[i] = acc;
            }
            // FP32 plans: which of the lane's sites hold a filter value at or above kRangeFloor
            uint32_t okb = 0;
            if (rsc.words) {
#pragma unroll
                for (int i = 0; i < 16; ++i) okb |= (ring[b][i] >= (T)kRangeFloor ? 1u : 0u) << i;
            }
            load_row(nd - s - NB, ring[b]);  // this buffer now serves draw s + NB
            const double tot = P[15] * gy;
            double total;
            const double incl = wave_incl_scan_f64(tot, lane, &total);
            int chosen = cur;
            bool low = false;  // FP32: drawn from a filter value below kRangeFloor, or no weight
            if (!(total > 0.0) || !isfinite(total)) {
                if (rsc.words)
                    low = true;
                else if (real && err == 0)
                    err = isfinite(total) ? FH_ERR_ZERO_WEIGHT : FH_ERR_NONFINITE;
            } else {
                const double T_ = u * total;
                const double Tl = fmax((T_ - (incl - tot)) / gy, 0.0);
                int cnt = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) cnt += P[i] <= Tl ? 1 : 0;
                const uint64_t found = __ballot(tot > 0.0 && cnt < 16);
                if (found) {
                    const int src = __ffsll((unsigned long long)found) - 1;
                    const int k = __builtin_amdgcn_readlane(cnt, src);
                    chosen = 16 * src + k;
                    low = ((__builtin_amdgcn_readlane((int)okb, src) >> k) & 1) == 0;
                } else {
                    int lastpos = -1;
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (gy > 0.0 && P[i] > (i ? P[i - 1] : 0.0)) lastpos = i;
                    const uint64_t has = __ballot(lastpos >= 0);
                    if (has) {
                        const int src = 63 - __clzll((long long)has);
                        const int k = __builtin_amdgcn_readlane(lastpos, src);
                        chosen = 16 * src + k;
                        low = ((__builtin_amdgcn_readlane((int)okb, src) >> k) & 1) == 0;
                    }
                }
                low = low && rsc.words;
            }
            if (low && real) {
                halted = true;  // an FP32 value near FP32's floor decides it: FP64 redraw
                if (lane == 0) rescue_push(rsc, c, t.chain, t.p, t.block, kCauseDraw);
            }
            chosen = real ? chosen : cur;
            pc[(int64_t)((start + j) % L_tau) * c.np + (start + j >= L_tau ? qn : t.p)] = chosen;
            cur = chosen;
        }
    }
    if (err != 0 && lane == 0) set_status(status, err, t.chain);  // the block's first error
}

// Inclusive scan within a DPP row of 16 lanes.
__device__ inline double group_scan_incl(double v) {
    v += dpp_f64<0x111>(v);
    v += dpp_f64<0x112>(v);
    v += dpp_f64<0x114>(v);
    v += dpp_f64<0x118>(v);
    return v;
}

// Full-row draw by the whole wavefront for one group's worldline (the draw rule of k_backward:
// the first site in site order whose cumulative weight exceeds u times the total, else the last
// site with a positive weight). Lane k owns the per = ceil(N / 64) contiguous sites from k per;
// the weights max(f, 0) g(dy) g(dx) are taken about (cx, cy). Every argument is wavefront
// uniform. On a zero or non-finite total the current site is kept and *bad gets the error;
// with `range` (FP32 plans) such a total, or a drawn site whose filter value is below
// kRangeFloor, sets *bad = kBadRange instead.
constexpr int kBadRange = 1;
template <typename T>
__device__ int wave_row_draw(const T* __restrict__ row, int N, int L, int cx, int cy,
                             const double* g, double u, int cur, int lane, int* bad,
                             bool range = false) {
    constexpr int C = 8;  // loads in flight per lane (register budget of the caller)
    const int per = (N + 63) >> 6;
    const int i0 = lane * per;
    const int cnt = max(0, min(per, N - i0));
    auto weight = [&](T fv, int x, int y) {
        int dx = cx - x, dy = cy - y;
        dx += dx < 0 ? L : 0;
        dy += dy < 0 ? L : 0;
        const double f = (double)fv;
        return (f > 0.0 ? f : 0.0) * (g[dy] * g[dx]);
    };
    const int x0 = cnt > 0 ? i0 % L : 0, y0 = cnt > 0 ? i0 / L : 0;
    double tot = 0.0;
    int lastpos = -1;
    {
        int x = x0, y = y0;
#pragma unroll 1
        for (int m0 = 0; m0 < cnt; m0 += C) {
            T v[C];
#pragma unroll
            for (int k = 0; k < C; ++k) v[k] = row[min(i0 + m0 + k, N - 1)];
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (m0 + k < cnt) {
                    const double w = weight(v[k], x, y);
                    tot += w;
                    if (w > 0.0) lastpos = i0 + m0 + k;
                    if (++x == L) {
                        x = 0;
                        ++y;
                    }
                }
        }
    }
    double total;
    const double incl = wave_incl_scan_f64(tot, lane, &total);
    if (range && (!(total > 0.0) || !isfinite(total))) {
        *bad = kBadRange;
        return cur;
    }
    if (!(total > 0.0) || !isfinite(total)) {
        *bad = isfinite(total) ? FH_ERR_ZERO_WEIGHT : FH_ERR_NONFINITE;
        return cur;
    }
    const double Tq = u * total;
    const uint64_t fm = __ballot(incl > Tq && tot > 0.0);
    if (fm) {
        const int src = __ffsll((unsigned long long)fm) - 1;
        int pick = -1;
        if (lane == src) {  // the lane holding the crossing walks its sites again
            double run = incl - tot;
            int x = x0, y = y0, last_in = -1;
#pragma unroll 1
            for (int m0 = 0; m0 < cnt && pick < 0; m0 += C) {
                T v[C];
#pragma unroll
                for (int k = 0; k < C; ++k) v[k] = row[min(i0 + m0 + k, N - 1)];
#pragma unroll
                for (int k = 0; k < C; ++k)
                    if (m0 + k < cnt && pick < 0) {
                        const double w = weight(v[k], x, y);
                        run += w;
                        if (w > 0.0) last_in = i0 + m0 + k;
                        if (run > Tq) pick = i0 + m0 + k;
                        if (++x == L) {
                            x = 0;
                            ++y;
                        }
                    }
            }
            if (pick < 0) pick = last_in >= 0 ? last_in : lastpos;  // rounding between orders
        }
        const int chosen = __builtin_amdgcn_readlane(pick, src);
        if (range && !((double)row[chosen] >= kRangeFloorD)) *bad = kBadRange;
        return chosen;
    }
    const uint64_t lm = __ballot(lastpos >= 0);
    const int chosen = lm ? __builtin_amdgcn_readlane(lastpos, 63 - __clzll((long long)lm)) : cur;
    if (range && !((double)row[chosen] >= kRangeFloorD)) *bad = kBadRange;
    return chosen;
}

// Draw on the window of half-width w <= kWin2W around (cx, cy), taken by the whole wavefront:
// lane k holds the window ranks 4k .. 4k + 3 (site order), so the draw costs one round trip of
// four loads per lane. The lane sums are scanned across the wavefront and the lane holding the
// first rank above tau certifies the draw against `bound` (the outside bound times the row's mass
// bound, fh_window.h). Every argument is wavefront uniform.
// Returns (1 << 16 | y << 8 | x) for a certified draw, 0 otherwise (uniform); *fsel receives
// the drawn site's filter value.
template <typename T>
__device__ int wave_window_draw(const T* __restrict__ row, int L, int cx, int cy, int w,
                                const double* g, double u, double bound, int lane,
                                double* fsel) {
    constexpr int K = 4;
    static_assert(64 * K >= (2 * kWin2W + 1) * (2 * kWin2W + 1), "the window fits the wavefront");
    const int WW = win_width(w, L), nwin = WW * WW;
    const float rw = 1.0f / (float)WW;  // (q + 1/2) / WW in FP32 floors exactly for q < 2^12
    int tx, bx, ty, by;
    win_axis(cx, w, L, WW, &tx, &bx);
    win_axis(cy, w, L, WW, &ty, &by);
    int xs[K], ys[K];
    T fv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = lane * K + k;
        const int qq = q < nwin ? q : 0;
        const int qy = (int)(((float)qq + 0.5f) * rw);
        xs[k] = win_at(qq - qy * WW, tx, bx);
        ys[k] = win_at(qy, ty, by);
        fv[k] = row[ys[k] * L + xs[k]];
    }
    double P[K];
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int dx = cx - xs[k], dy = cy - ys[k];
        dx += dx < 0 ? L : 0;
        dy += dy < 0 ? L : 0;
        const double f = lane * K + k < nwin ? (double)fv[k] : 0.0;
        acc += (f > 0.0 ? f : 0.0) * (g[dy] * g[dx]);
        P[k] = acc;
    }
    double T_in;
    const double incl = wave_incl_scan_f64(acc, lane, &T_in);
    const double excl = incl - acc;
    const double tau = u * T_in;
    const bool fin = T_in > 0.0 && isfinite(T_in);
    const uint64_t fm = __ballot(fin && incl > tau && acc > 0.0);
    if (!fm) return 0;
    const int src = __ffsll((unsigned long long)fm) - 1;
    int res = 0;
    double fp = 0.0;
    if (lane == src) {
        double c_lo = excl, c_hi = 0.0;
        int pick = -1, pxy = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double ck = excl + P[k];
            if (pick < 0) {
                if (ck > tau) {
                    pick = k;
                    pxy = xs[k] | (ys[k] << 8);
                    c_hi = ck;
                    fp = (double)fv[k];
                } else {
                    c_lo = ck;
                }
            }
        }
        if (pick >= 0 && win_certified(c_lo, c_hi, tau, bound + kWinSlack * T_in))
            res = (1 << 16) | pxy;
    }
    *fsel = readlane_f64(fp, src);
    return __builtin_amdgcn_readlane(res, src);
}

// Backward sampling with windowed draws (the certificate is in fh_window.h): 16 lanes per
// (chain, worldline, block), four per wavefront, so that every wavefront keeps four independent
// chains of dependent loads in flight. Lane li holds the window ranks 4 li .. 4 li + 3 (site
// order). Per draw it loads those filter values, forms max(f, 0) g(dy) g(dx), and the 16 lanes
// scan their sums with DPP inside their row of the wavefront. The lane holding the first rank
// above tau certifies the draw. An uncertified draw is retried on the wider window, and failing
// that on the row in site order with k_backward's rule; the whole wavefront takes each of these,
// one such group at a time (four window ranks, or ceil(N / 64) contiguous sites, per lane).
// Lane li of a group computes
// the Philox uniform of draw s0 + li once per 16 draws. Every load address is in bounds for any
// lane (inactive groups read chain 0's first row), so loads are unconditional and values masked.
// SLOT (T = double): the draws of phase A of the FP64 re-filter, the held chains' blocks in the
// queue's phase A part, from their representatives' FP64 rows in the re-filter's slots (windowed
// chains; k_rescue_share_draw takes the others). The rule is the FP64 plans', so the sites equal
// those of k_rescue's draws; a worldline that shares its representative's rows also gets its
// log Z from the representative's end tile.
template <typename T, bool SLOT = false>
__global__ __launch_bounds__(kThreads) void k_backward_win(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const double* __restrict__ tables, const T* __restrict__ filt, int32_t* __restrict__ paths,
    const int32_t* __restrict__ perm, const uint64_t* __restrict__ sweep_ptr, int32_t* status,
    int32_t* __restrict__ bw_state, int count_uncertified, const Rescue rsc, const SlotRows sr) {
    static_assert(!SLOT || sizeof(T) == 8, "phase A's rows are FP64");
    constexpr int G = kThreads / kWinLanes;
    constexpr int K = kWinPerLane;
    // g(d) for d in (-L, L): gsh[grp][kWinMaxL + d], so a signed offset indexes it directly
    __shared__ double gsh[G][2 * kWinMaxL];
    const int grp = threadIdx.x / kWinLanes, li = threadIdx.x % kWinLanes;
    const int lane64 = threadIdx.x & 63;
    const int gbase = lane64 - li;  // the group's first lane in the wavefront
    const int task = blockIdx.x * G + grp;
    // while the plan is on the full-row kernels, they draw these tasks
    const bool listed = SLOT ? task < rsc.words[3] : task < n_tasks && bw_state[0] == 0;
    const DrawTask t = listed ? (SLOT ? rsc.list[task] : tasks[task]) : DrawTask{0, 0, 0, 0};
    const ChainInfo& c = chains[t.chain];
    // a block queued for the FP64 re-filter is drawn by k_rescue (SLOT: by this kernel when its
    // chain is windowed)
    const bool active = SLOT ? listed && c.win_on : listed && !rescue_queued(rsc, c, t.p, t.block);
    // an inactive group draws nothing; on a one-site lattice its table fill and loads stay minimal
    const int L = active ? c.L : 1, N = active ? c.N : 1, L_tau = c.L_tau, w = c.win_w;
    double* g = gsh[grp] + kWinMaxL;  // g[d] = g(d mod L) for -L < d < L
    for (int d = li; d < L; d += kWinLanes) {
        const double gd = tables[tab_g(c) + d];
        g[d] = gd;
        g[d - L] = gd;
    }
    __syncthreads();  // the only barrier; every wave reaches it
    const uint64_t sweep = *sweep_ptr;
    int start = 0, len = 1;
    if (active) block_of(c, sweep, t.block, &start, &len);
    const int nd = len - 1;  // draw s sets slice start + (nd - s), s = 0 .. nd - 1
    int nd_max = nd;
    nd_max = max(nd_max, __shfl_xor(nd_max, 16, 64));
    nd_max = max(nd_max, __shfl_xor(nd_max, 32, 64));
    int32_t* pc = paths + c.path_off;
    const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
    int cur = 0;
    if (nd >= 1)
        cur = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                              (start + len >= L_tau ? qn : t.p)], N, status, t.chain);
    int cx = cur % L, cy = cur / L;
    const int WW = win_width(w, L), nwin = WW * WW;
    int qx[K], qy[K];
    bool qv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = li * K + k;
        qv[k] = q < nwin;
        qy[k] = qv[k] ? q / WW : 0;
        qx[k] = qv[k] ? q - qy[k] * WW : 0;
    }
    const int ro = row_owner(rsc, c, t.p, t.block);  // shared forward filters
    const int64_t ri = c.blk_off + (int64_t)ro * c.nb + t.block;
    const T* rows;
    if constexpr (SLOT)  // the representative's slot (inactive groups read slot 0)
        rows = (const T*)(sr.ws + (active ? (int64_t)sr.rep_slot[ri] * sr.slot_elems : 0));
    else
        rows = filt + c.filt_off + ((int64_t)ro * L_tau + (int64_t)t.block * (c.B - 1)) * N;
    // the outside bound scales with the row mass (2^row_exp on FP32 plans; phase A's FP64 rows
    // are normalised)
    const double mass = SLOT ? 1.0 : c.row_mass;
    const double gout = c.win_gout * mass * kWinMassBound;
    double ureg = 0.0;
    int err = 0;  // the first error of the block, reported once after the loop
    int n_unc = 0;  // draws the first window did not certify (kept by lane 0 of the group)
    // Drawn sites are stored sixteen draws at a time: lane li keeps the site of draw sb + li of
    // the current batch sb. A store retires in order with the loads after it, so a store after
    // every draw would make each draw's window loads wait for the previous draw's store; the
    // batch store is issued after the next draw's loads.
    int pend = 0;
    bool halt = false;  // the block left FP32's range: k_rescue redraws it
    auto flush = [&](int sb) {
        const int sd = sb + li;
        if (sd < nd) {
            const int jd = nd - sd;
            pc[(int64_t)((start + jd) % L_tau) * c.np + (start + jd >= L_tau ? qn : t.p)] = pend;
        }
    };
    for (int s = 0; s < nd_max; ++s) {
        const bool real = s < nd && !halt;
        const int j = s < nd ? nd - s : 1;
        if ((s & 15) == 0) {  // lane li draws the uniform of draw s + li
            const int jj = nd - s - li;
            ureg = 0.0;
            if (jj >= 1) {
                const u64x4 r = philox4x64_10((uint64_t)t.p, (uint64_t)((start + jj) % L_tau),
                                              sweep, kTagPath, c.seed, 0);
                ureg = u01_from(r.x0);
            }
        }
        const double u = __shfl(ureg, gbase + (s & 15), 64);
        const T* row = rows + (int64_t)(j - 1) * N;
        int xs[K], ys[K];
        T fv[K];
        int tx, bx, ty, by;
        win_axis(cx, w, L, WW, &tx, &bx);
        win_axis(cy, w, L, WW, &ty, &by);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            xs[k] = win_at(qx[k], tx, bx);
            ys[k] = win_at(qy[k], ty, by);
            fv[k] = row[ys[k] * L + xs[k]];
        }
        __builtin_amdgcn_sched_barrier(0);
        if ((s & 15) == 0 && s > 0) flush(s - 16);  // the previous batch, after these loads
        __builtin_amdgcn_sched_barrier(0);
        double P[K];
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int dx = cx - xs[k], dy = cy - ys[k];  // in (-L, L)
            // max(f, 0) of the window's filter values (0 off the window and for NaN), selected
            // in the rows' own precision
            const T fk = (real && qv[k] && fv[k] > T(0)) ? fv[k] : T(0);
            acc += (double)fk * (g[dy] * g[dx]);
            P[k] = acc;
        }
        double incl = acc;  // inclusive scan over the group's 16 lanes (one DPP row)
        incl += dpp_f64<0x111>(incl);
        incl += dpp_f64<0x112>(incl);
        incl += dpp_f64<0x114>(incl);
        incl += dpp_f64<0x118>(incl);
        const double excl = dpp_f64<0x111>(incl);  // the previous lane's inclusive sum (0 first)
        const double T_in = dpp_f64<0x15F>(incl);  // row_newbcast:15, the group's total
        const double tau = u * T_in;
        const bool fin = T_in > 0.0 && isfinite(T_in);
        const uint32_t gm =
            (uint32_t)(__ballot(real && fin && incl > tau && acc > 0.0) >> gbase) & 0xFFFFu;
        const int src = gm ? __ffs((int)gm) - 1 : 0;
        // The lane's cumulative sums E[k + 1] = excl + P[k] rise with k (nonnegative terms,
        // monotone rounding), so the first rank whose sum exceeds tau is the number of sums not
        // above it (K: none); the bracket (E[pick], E[pick + 1]) and the site follow from it by
        // a two-level select (K = 4).
        static_assert(K == 4, "the selects below take four ranks");
        double E[K + 1];
        E[0] = excl;
        int pick = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            E[k + 1] = excl + P[k];
            pick += E[k + 1] > tau ? 0 : 1;
        }
        const bool q1 = (pick & 2) != 0, q0 = (pick & 1) != 0;
        auto sel = [&](auto a0, auto a1, auto a2, auto a3) {
            return q1 ? (q0 ? a3 : a2) : (q0 ? a1 : a0);
        };
        const double c_lo = sel(E[0], E[1], E[2], E[3]), c_hi = sel(E[1], E[2], E[3], E[4]);
        const int px = sel(xs[0], xs[1], xs[2], xs[3]), py = sel(ys[0], ys[1], ys[2], ys[3]);
        const double fp = (double)sel(fv[0], fv[1], fv[2], fv[3]);
        const bool cert_l = li == src && pick < K &&
                            win_certified(c_lo, c_hi, tau, gout + kWinSlack * T_in);
        // the source lane's draw to its group: only that lane contributes to an OR scan over
        // the group's DPP row, whose last lane then broadcasts it (no LDS round trip). Bit 17:
        // the drawn site's filter value is below kRangeFloor (FP32 plans redraw it in FP64).
        int mine = li == src ? (cert_l ? 1 << 16 : 0) | (!(fp >= kRangeFloorD) ? 1 << 17 : 0) |
                                   (py << 8) | px
                             : 0;
        mine |= __builtin_amdgcn_mov_dpp(mine, 0x111, 0xF, 0xF, true);  // row_shr:1
        mine |= __builtin_amdgcn_mov_dpp(mine, 0x112, 0xF, 0xF, true);  // row_shr:2
        mine |= __builtin_amdgcn_mov_dpp(mine, 0x114, 0xF, 0xF, true);  // row_shr:4
        mine |= __builtin_amdgcn_mov_dpp(mine, 0x118, 0xF, 0xF, true);  // row_shr:8
        const int packed = __builtin_amdgcn_mov_dpp(mine, 0x15F, 0xF, 0xF, false);
        const bool cert = gm != 0 && ((packed >> 16) & 1) != 0;
        if (!SLOT && rsc.words && real && cert && ((packed >> 17) & 1)) halt = true;
        int nx = packed & 255, ny = (packed >> 8) & 255;
        bool need_row = false;
        n_unc += (real && !cert) ? 1 : 0;
        // an uncertified draw tries the wider window, one such group at a time, taken by the
        // whole wavefront
        uint64_t wide_left = __ballot(li == 0 && real && !cert);
        while (wide_left) {
            const int g0 = __ffsll((unsigned long long)wide_left) - 1;  // the group's lane 0
            wide_left &= wide_left - 1;
            const uint64_t rp = (uint64_t)(uintptr_t)row;
            const T* rowg = (const T*)(uintptr_t)(
                (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)rp, g0) |
                ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(rp >> 32), g0) << 32));
            double f2;
            const int p2 = wave_window_draw(
                rowg, __builtin_amdgcn_readlane(L, g0), __builtin_amdgcn_readlane(cx, g0),
                __builtin_amdgcn_readlane(cy, g0), kWin2W,
                gsh[(threadIdx.x >> 6) * 4 + (g0 >> 4)] + kWinMaxL, readlane_f64(u, g0),
                readlane_f64(c.win_gout2 * mass * kWinMassBound, g0), lane64, &f2);
            if ((lane64 >> 4) == (g0 >> 4)) {
                if (p2 >> 16) {
                    nx = p2 & 255;
                    ny = (p2 >> 8) & 255;
                    if (!SLOT && rsc.words && !(f2 >= kRangeFloorD)) halt = true;
                } else {
                    need_row = true;
                }
            }
        }
        // then the full row, one group at a time, by the whole wavefront
        uint64_t rows_left = __ballot(li == 0 && need_row);
        while (rows_left) {
            const int g0 = __ffsll((unsigned long long)rows_left) - 1;  // the group's lane 0
            rows_left &= rows_left - 1;
            const uint64_t rp = (uint64_t)(uintptr_t)row;
            const T* rowg = (const T*)(uintptr_t)(
                (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)rp, g0) |
                ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(rp >> 32), g0) << 32));
            int bad = 0;
            const int Lg = __builtin_amdgcn_readlane(L, g0);
            const int chosen = wave_row_draw(
                rowg, __builtin_amdgcn_readlane(N, g0), Lg, __builtin_amdgcn_readlane(cx, g0),
                __builtin_amdgcn_readlane(cy, g0), gsh[(threadIdx.x >> 6) * 4 + (g0 >> 4)] + kWinMaxL,
                readlane_f64(u, g0), __builtin_amdgcn_readlane(cur, g0), lane64, &bad,
                !SLOT && rsc.words != nullptr);
            if ((lane64 >> 4) == (g0 >> 4)) {
                nx = chosen % Lg;
                ny = chosen / Lg;
                if (bad == kBadRange)
                    halt = true;
                else if (bad != 0 && err == 0)
                    err = bad;
            }
        }
        if (real) {
            cx = nx;
            cy = ny;
            cur = cx + L * cy;
        }
        if (li == (s & 15)) pend = cur;
    }
    if (nd_max > 0) flush((nd_max - 1) & ~15);
    if (halt && li == 0) rescue_push(rsc, c, t.chain, t.p, t.block, kCauseDraw);
    if (err != 0 && li == 0) set_status(status, err, t.chain);  // the block's first error
    if (count_uncertified && active && li == 0 && n_unc > 0)
        atomicAdd(&bw_state[kBwCounts + t.chain], n_unc);
    if constexpr (SLOT) {  // a worldline sharing its representative's rows: its own end weight
        if (active && li == 0 && ro != t.p) {
            const int e = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                                          (start + len >= L_tau ? qn : t.p)], N, status, t.chain);
            const double hv = (double)rows[(int64_t)(c.B - 1) * N + e];  // the end tile
            if (!(hv > 0.0)) set_status(status, FH_ERR_NONFINITE, t.chain);
            sr.blk_logz[c.blk_off + (int64_t)t.p * c.nb + t.block] = sr.blk_la[ri] + log(hv);
        }
    }
}

// The draws of one re-filtered block from its FP64 rows, by the whole wavefront: the rule of
// the FP64 plans' backward kernels, taken on the certified window of half-width win_w, else on
// the wider one, else on the full row (fh_window.h), so the sites are those of an FP64 plan.
// Kept out of line: inlined into k_rescue next to the FP64 forward recursion, the compiler fails.
// CTX tells the callers apart, so that each copy is compiled for its caller's register budget.
template <int CTX>
__device__ __attribute__((noinline)) void rescue_draws(const DrawTask& t, const ChainInfo& c,
                                                       const double* g, int32_t* paths,
                                                       const int32_t* perm, uint64_t sweep,
                                                       int32_t* status, int lane,
                                                       const double* rows) {
    int start, len;
    block_of(c, sweep, t.block, &start, &len);
    if (len < 2) return;
    const int L = c.L, N = c.N, L_tau = c.L_tau;
    int32_t* pc = paths + c.path_off;
    const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
    int cur = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                              (start + len >= L_tau ? qn : t.p)], N, status, t.chain);
    int err = 0;
    // Draw s sets slice start + (nd - s). Uniforms are made 64 draws at a time (lane k that of
    // draw s + k) and drawn sites stored 64 at a time (lane k keeps that of draw s + k): a
    // store per draw would make each draw's window loads wait for it (loads and stores retire
    // in order), and a Philox evaluation per draw would sit on the chain of dependent draws.
    const int nd = len - 1;
    double ureg = 0.0;
    int pend = 0;
    auto flush = [&](int sb) {
        const int sd = sb + lane;
        if (sd < nd) {
            const int jd = nd - sd;
            pc[(int64_t)((start + jd) % L_tau) * c.np + (start + jd >= L_tau ? qn : t.p)] = pend;
        }
    };
    for (int s = 0; s < nd; ++s) {
        const int j = nd - s;
        if ((s & 63) == 0) {
            if (s > 0) flush(s - 64);
            const int jj = j - lane;
            ureg = 0.0;
            if (jj >= 1)
                ureg = u01_from(philox4x64_10((uint64_t)t.p, (uint64_t)((start + jj) % L_tau),
                                              sweep, kTagPath, c.seed, 0).x0);
        }
        const double u = readlane_f64(ureg, s & 63);
        const double* row = rows + (int64_t)(j - 1) * N;
        const int cx = cur % L, cy = cur / L;
        int site = -1;
        double f;
        if (c.win_on) {
            int pk = wave_window_draw(row, L, cx, cy, c.win_w, g, u, c.win_gout * kWinMassBound,
                                      lane, &f);
            if (!(pk >> 16))
                pk = wave_window_draw(row, L, cx, cy, kWin2W, g, u, c.win_gout2 * kWinMassBound,
                                      lane, &f);
            if (pk >> 16) site = (pk & 255) + L * ((pk >> 8) & 255);
        }
        if (site < 0) {
            int bad = 0;
            site = wave_row_draw(row, N, L, cx, cy, g, u, cur, lane, &bad);
            if (bad != 0 && err == 0) err = bad;
        }
        if (lane == (s & 63)) pend = site;
        cur = site;
    }
    if (nd > 0) flush((nd - 1) & ~63);
    if (err != 0 && lane == 0) set_status(status, err, t.chain);
}

// FP64 re-filter and redraw of the blocks an FP32 pass queued because their filters left
// FP32's range (kRangeFloor). The FP32 pass's rows for such a block hold values at FP32's floor
// that decide its draws and log Z; FP64 holds them to ~2^-1022. Phase 0 takes the whole queue,
// phase 1 its phase A [0, words[3]) (a sweep's held chains, beside the FP32 passes), phase 2 the
// rest (after phase 1 has ended). One wavefront takes queued blocks i = lo + wid,
// lo + wid + n_slots, ... in turn, with its own slot of FP64 rows:
//   forward: the block recursion of k_forward_dmfma on the FP64 circulant, with the FP64
//            W~ = exp(coef aux - m_l) of k_rescue_potentials (the FP32 tables may hold zeros
//            there); log Z to blk_logz; rows to the slot (DRAW), or else, rounded and scaled,
//            to the plan's FP32 rows (what fh_get_filters returns after fh_forward_filter);
//   DRAW:    the block's sites from the slot's rows with k_backward's full-row rule and the same
//            Philox uniforms, so the draws are those of an FP64 plan.
// NT = 2 takes the chains with L <= 32; NT = 3 and 4 the 48 x 48 and 64 x 64 chains (one
// wavefront per SIMD: their tiles take 256 registers), each launch skipping the other chains'
// blocks. A queued block of a lattice without the FP64 circulant (fp64_circulant) latches
// FH_ERR_NONFINITE and keeps its sites. Every wavefront reads the queue length once and leaves
// when its share is done.
template <bool DRAW, int NT>
__global__ __launch_bounds__(kThreads, NT == 2 ? 2 : 1) void k_rescue(
    const ChainInfo* __restrict__ chains, const double* __restrict__ tables,
    const double* __restrict__ cmat64, const float* __restrict__ aux,
    const double* __restrict__ wshift, int64_t total_slices, int32_t* __restrict__ paths,
    const int32_t* __restrict__ perm, float* __restrict__ filt, double* __restrict__ blk_logz,
    const uint64_t* __restrict__ sweep_ptr, int32_t* status, const Rescue rsc,
    double* __restrict__ ws, int64_t slot_elems, int n_slots, const double* __restrict__ W64,
    int64_t aux_elems, int phase) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    // phase 1 reads only words[3]: the FP32 passes beside it still append to the queue
    const int lo = phase == 2 ? __builtin_amdgcn_readfirstlane(rsc.words[3]) : 0;
    const int hi = __builtin_amdgcn_readfirstlane(rsc.words[phase == 1 ? 3 : 0]);
    if (NT == 2 && DRAW && wid == 0 && lane == 0 && hi > lo) atomicAdd(&rsc.words[1], hi - lo);
    double* slot = ws + (int64_t)wid * slot_elems;
    const uint64_t sweep = *sweep_ptr;
    for (int i = lo + wid; i < hi; i += n_slots) {
        const DrawTask t = rsc.list[i];
        const ChainInfo& c = chains[t.chain];
        if (NT == 2 ? c.L > 32 : c.L != 16 * NT) {  // another launch's chain, or none's
            if (NT == 2 && !fp64_circulant(c.L) && lane == 0)
                set_status(status, FH_ERR_NONFINITE, t.chain);
            continue;
        }
        int start, len;
        block_of(c, sweep, t.block, &start, &len);
        // the 48 x 48 and 64 x 64 tilings take L as a constant (their site offsets fold into
        // the stores' immediates instead of taking registers)
        const int L = NT == 2 ? c.L : 16 * NT, N = NT == 2 ? c.N : 256 * NT * NT, L_tau = c.L_tau;
        const int spin = t.p >= c.n_up ? 1 : 0;
        const double coef = spin ? c.coef_dn : c.coef_up;
        const double* shift = wshift + spin * total_slices + c.slice_off;
        const float* ax = aux + c.aux_off;
        int32_t* pc = paths + c.path_off;
        const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
        const int a = checked_site(pc[(int64_t)start * c.np + t.p], N, status, t.chain);
        const int e = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                                      (start + len >= L_tau ? qn : t.p)], N, status, t.chain);
        double Cb[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) Cb[q] = cmat64[((int64_t)t.chain * 16 + q) * 64 + lane];
        float* frows = filt + c.filt_off + ((int64_t)t.p * L_tau + (int64_t)t.block * (c.B - 1)) * N;
        const double* Wl0 = W64 + spin * aux_elems + c.aux_off;
        // the site of the lane's element (q, r) of the tiling; padded positions (L < 32) read
        // W at site 0, times an exact zero, and store nothing
        auto site = [&](int q, int r) {
            if constexpr (NT == 2) {
                const int x = t64_x(q, lane), y = t64_y(q, r, lane);
                return (x < L && y < L) ? y * L + x : -1;
            } else {
                return tb_y<NT>(q, r, lane) * L + tb_x<NT>(q, lane);
            }
        };
        auto wtab = [&](int l, auto& w) {
            const double* Wl = Wl0 + (int64_t)l * N;
#pragma unroll
            for (int q = 0; q < (NT == 2 ? 4 : NT * NT); ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) w[4 * q + r] = Wl[max(site(q, r), 0)];
        };
        auto put = [&](int j, int q, int r, double v) {
            const int64_t o = (int64_t)(j - 1) * N + site(q, r);
            if (DRAW)
                slot[o] = v;                         // the rows the draws below read
            else
                frows[o] = (float)(v * c.row_mass);  // the plan's rows (FP32 scaling)
        };
        bool ok = true;
        const double la0 = coef * (double)ax[(int64_t)start * N + a];
        double lz;
        if constexpr (NT == 2) {
            lz = dmfma_block_forward(Cb, L, L_tau, start, len, a, e, la0, shift, wtab, put, &ok);
        } else {
            double la_end;
            lz = dmfma_big_block_forward_end<NT>(Cb, L_tau, start, len, a, e, la0, shift, wtab,
                                                 put, [](int, int, double) {}, &la_end, &ok);
        }
        if (lane == 0) {
            if (!ok) set_status(status, FH_ERR_NONFINITE, t.chain);
            blk_logz[c.blk_off + (int64_t)t.p * c.nb + t.block] = lz;
        }
        if (!DRAW || !ok) continue;
        // the slot's rows were stored by this wavefront's lanes: make them visible to its loads
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        // the full-row rule of the FP64 plans' backward kernel, on the slot's rows
        rescue_draws<0>(t, c, tables + tab_g(c), paths, perm, sweep, status, lane, slot);
        // the next block reuses the slot: its stores must follow these loads
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    }
}

// Phase A of the FP64 re-filter (the held chains, beside the FP32 passes), first kernels: the
// forward recursion of each representative in the dense list arep (k_rescue_held; every block
// of a chain without shared filters), into a slot of its own (k_rescue_held admitted only
// chains whose recursions fit the slots): the rows, then the end tile C f~ C. The block's log Z
// goes to blk_logz, log Z without the end weight to blk_la (shared-filter chains), and the slot
// to rep_slot.
//
// Lattices with L <= 32: one workgroup of four wavefronts per representative. Wavefront q owns
// the 16 x 16 tile q = 2 I + J of the padded 32 x 32 filter (fh_dmfma.h): every wavefront holds
// the whole filter F, forms the two tiles X(0, I), X(1, I) of X = F^T C that its tile of
// H = X^T C needs, then that tile: 24 products per step where one wavefront takes 64. The four
// W-weighted tiles meet in LDS, and every wavefront sums all of them in the order of
// dmfma_block_forward_end, so the normaliser, the rows, the end tile and log Z are bit for bit
// those of the one-wavefront recursion (k_rescue).
__global__ __launch_bounds__(kThreads, 1) void k_rescue_share_fwd4(
    const ChainInfo* __restrict__ chains, const double* __restrict__ cmat64,
    const float* __restrict__ aux, const double* __restrict__ wshift, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm,
    double* __restrict__ blk_logz, double* __restrict__ blk_la,
    const uint64_t* __restrict__ sweep_ptr, int32_t* status, const Rescue rsc,
    const DrawTask* __restrict__ arep, int32_t* __restrict__ rep_slot, double* __restrict__ ws,
    int64_t slot_elems, const double* __restrict__ W64, int64_t aux_elems) {
    static_assert(kWaves == 4, "one wavefront per 16 x 16 tile of the 32 x 32 filter");
    __shared__ f64x4 xch[2][4][64];  // the W-weighted tiles of a step, double-buffered
    __shared__ int32_t slot_sh;
    const int lane = threadIdx.x & 63;
    const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // this wavefront's tile
    const int I = wq >> 1, J = wq & 1;
    const int n = __builtin_amdgcn_readfirstlane(rsc.words[6]);
    const uint64_t sweep = *sweep_ptr;
    int buf = 0;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const DrawTask t = arep[i];
        const ChainInfo& c = chains[t.chain];
        if (c.L > 32) continue;  // the 16 x 16 tilings take it (the whole workgroup skips)
        if (threadIdx.x == 0) slot_sh = atomicAdd(&rsc.words[4], 1);
        __syncthreads();
        const int slot_id = slot_sh;
        double* slot = ws + (int64_t)slot_id * slot_elems;
        int start, len;
        block_of(c, sweep, t.block, &start, &len);
        const int L = c.L, N = c.N, L_tau = c.L_tau;
        const int spin = t.p >= c.n_up ? 1 : 0;
        const double coef = spin ? c.coef_dn : c.coef_up;
        const double* shift = wshift + spin * total_slices + c.slice_off;
        const int32_t* pc = paths + c.path_off;
        const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
        const int a = checked_site(pc[(int64_t)start * c.np + t.p], N, status, t.chain);
        const int e = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                                      (start + len >= L_tau ? qn : t.p)], N, status, t.chain);
        // the B operands this wavefront's products take: column block I of C for X(K, I),
        // column block J for its tile of H (loaded by index, not picked from registers at a
        // run-time index, which would put them in scratch)
        double CbI[8], CbJ[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            CbI[k] = cmat64[((int64_t)t.chain * 16 + k * 2 + I) * 64 + lane];
            CbJ[k] = cmat64[((int64_t)t.chain * 16 + k * 2 + J) * 64 + lane];
        }
        const double* Wl0 = W64 + spin * aux_elems + c.aux_off;
        // this wavefront's elements: site of register r of tile wq (-1 where padded; W is read
        // at site 0 there and multiplies an exact zero)
        int site[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int x = t64_x(wq, lane), y = t64_y(wq, r, lane);
            site[r] = (x < L && y < L) ? y * L + x : -1;
        }
        auto load_w = [&](int l, double (&w)[4]) {
            const double* Wl = Wl0 + (int64_t)l * N;
#pragma unroll
            for (int r = 0; r < 4; ++r) w[r] = Wl[max(site[r], 0)];
        };
        // this wavefront's tile of H = (F^T C)^T C = C F C
        auto own_tile = [&](const Tile64& F) {
            f64x4 X[2];
#pragma unroll
            for (int K = 0; K < 2; ++K) {
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int K2 = 0; K2 < 2; ++K2)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F.t[2 * K2 + K][r],
                                                                   CbI[4 * K2 + r], acc, 0, 0, 0);
                X[K] = acc;
            }
            f64x4 H = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int K = 0; K < 2; ++K)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    H = __builtin_amdgcn_mfma_f64_16x16x4f64(X[K][r], CbJ[4 * K + r], H, 0, 0, 0);
            return H;
        };
        Tile64 F;
        const int ax = a % L, ay = a / L;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                F.t[q][r] = (t64_x(q, lane) == ax && t64_y(q, r, lane) == ay) ? 1.0 : 0.0;
        double la = coef * (double)aux[c.aux_off + (int64_t)start * N + a];
        bool good = true;
        // W of the next slice loaded one step ahead, in two buffers that swap roles
        double wa[4], wb[4];
        load_w((start + 1) % L_tau, wa);
        auto step = [&](int j, const double (&w)[4], double (&wf)[4]) {
            const int l = (start + j) % L_tau;
            const f64x4 H = own_tile(F);
            load_w((l + 1) % L_tau, wf);  // the last step fetches a slice it does not use
            f64x4 P;
#pragma unroll
            for (int r = 0; r < 4; ++r) P[r] = H[r] * w[r];
            xch[buf][wq][lane] = P;
            __syncthreads();
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const f64x4 v = xch[buf][q][lane];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    F.t[q][r] = v[r];
                    sum += v[r];
                }
            }
            buf ^= 1;
            const double tot = wave_sum_f64(sum);
            good = good && tot > 0.0 && isfinite(tot);
            const double inv = 1.0 / tot;
            la += log(tot) + shift[l];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) F.t[q][r] *= inv;
            // this wavefront's tile of the row: its own products scaled as F.t[wq] (read from
            // the products it holds, as F.t[wq] at a run-time index would live in scratch)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (site[r] >= 0) slot[(int64_t)(j - 1) * N + site[r]] = P[r] * inv;
        };
        int j = 1;
        for (; j + 1 < len; j += 2) {
            step(j, wa, wb);
            step(j + 1, wb, wa);
        }
        if (j < len) step(j, wa, wb);
        // end weight (C f~ C)(e): the end tile, and the element at e from its tile's wavefront
        const f64x4 H = own_tile(F);
        double* end = slot + (int64_t)(c.B - 1) * N;  // after the longest block's rows
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (site[r] >= 0) end[site[r]] = H[r];
        const int ex = e % L, ey = e / L;
        if (wq == 2 * (ey >> 4) + (ex >> 4)) {
            const int re = (ey & 15) >> 2;
            double hv = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r == re) hv = H[r];
            hv = __shfl(hv, (ex & 15) + 16 * (ey & 3), 64);
            if (lane == 0) {
                const int64_t bi = c.blk_off + (int64_t)t.p * c.nb + t.block;
                if (!(good && hv > 0.0)) set_status(status, FH_ERR_NONFINITE, t.chain);
                blk_logz[bi] = la + log(hv);
                if (c.dedup) blk_la[bi] = la;
                rep_slot[bi] = slot_id;
            }
        }
        __syncthreads();  // slot_sh and the exchange buffers are free for the next representative
    }
}

// The 48 x 48 and 64 x 64 chains' representatives (NT = 3, 4, fh_dmfma.h), one wavefront each,
// wavefront w taking entries w, w + n_waves, ... of arep.
template <int NT>
__global__ __launch_bounds__(kThreads, 1) void k_rescue_share_fwd(
    const ChainInfo* __restrict__ chains, const double* __restrict__ cmat64,
    const float* __restrict__ aux, const double* __restrict__ wshift, int64_t total_slices,
    const int32_t* __restrict__ paths, const int32_t* __restrict__ perm,
    double* __restrict__ blk_logz, double* __restrict__ blk_la,
    const uint64_t* __restrict__ sweep_ptr, int32_t* status, const Rescue rsc,
    const DrawTask* __restrict__ arep, int32_t* __restrict__ rep_slot, double* __restrict__ ws,
    int64_t slot_elems, int n_waves, const double* __restrict__ W64, int64_t aux_elems) {
    static_assert(NT == 3 || NT == 4, "the 16 x 16 tilings");
    constexpr int L = 16 * NT, N = L * L;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    const int n = __builtin_amdgcn_readfirstlane(rsc.words[6]);
    const uint64_t sweep = *sweep_ptr;
    for (int i = wid; i < n; i += n_waves) {
        const DrawTask t = arep[i];
        const ChainInfo& c = chains[t.chain];
        if (c.L != L) continue;  // another launch's chain
        int slot_id = 0;
        if (lane == 0) slot_id = atomicAdd(&rsc.words[4], 1);
        slot_id = __builtin_amdgcn_readfirstlane(__shfl(slot_id, 0, 64));
        double* slot = ws + (int64_t)slot_id * slot_elems;
        int start, len;
        block_of(c, sweep, t.block, &start, &len);
        const int L_tau = c.L_tau;
        const int spin = t.p >= c.n_up ? 1 : 0;
        const double coef = spin ? c.coef_dn : c.coef_up;
        const double* shift = wshift + spin * total_slices + c.slice_off;
        const int32_t* pc = paths + c.path_off;
        const int qn = perm[c.part_off + t.p];  // the worldline slices >= L_tau belong to
        const int a = checked_site(pc[(int64_t)start * c.np + t.p], N, status, t.chain);
        const int e = checked_site(pc[(int64_t)((start + len) % L_tau) * c.np +
                                      (start + len >= L_tau ? qn : t.p)], N, status, t.chain);
        double Cb[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) Cb[q] = cmat64[((int64_t)t.chain * 16 + q) * 64 + lane];
        const double* Wl0 = W64 + spin * aux_elems + c.aux_off;
        auto site = [&](int q, int r) { return tb_y<NT>(q, r, lane) * L + tb_x<NT>(q, lane); };
        auto wtab = [&](int l, double (&w)[4 * NT * NT]) {
            const double* Wl = Wl0 + (int64_t)l * N;
#pragma unroll
            for (int q = 0; q < NT * NT; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) w[4 * q + r] = Wl[site(q, r)];
        };
        auto put = [&](int j, int q, int r, double v) {
            slot[(int64_t)(j - 1) * N + site(q, r)] = v;
        };
        double* end = slot + (int64_t)(c.B - 1) * N;  // after the longest block's rows
        auto put_end = [&](int q, int r, double v) { end[site(q, r)] = v; };
        bool ok = true;
        double la_end = 0.0;
        const double la0 = coef * (double)aux[c.aux_off + (int64_t)start * N + a];
        const double lz = dmfma_big_block_forward_end<NT>(Cb, L_tau, start, len, a, e, la0, shift,
                                                          wtab, put, put_end, &la_end, &ok);
        if (lane == 0) {
            const int64_t bi = c.blk_off + (int64_t)t.p * c.nb + t.block;
            if (!ok) set_status(status, FH_ERR_NONFINITE, t.chain);
            blk_logz[bi] = lz;
            if (c.dedup) blk_la[bi] = la_end;
            rep_slot[bi] = slot_id;
        }
    }
}

// Phase A, second kernel: the draws of every queued block, one wavefront per block, from its
// representative's slot (its own for a chain without shared filters), with the FP64 plans' rule
// (rescue_draws); a block that shares rows also takes its log Z from the representative's log Z
// without the end weight and the end tile at its own end site.
__global__ __launch_bounds__(kThreads, kShareDrawWaves) void k_rescue_share_draw(
    const ChainInfo* __restrict__ chains, const double* __restrict__ tables,
    int32_t* __restrict__ paths, const int32_t* __restrict__ perm,
    double* __restrict__ blk_logz, const double* __restrict__ blk_la,
    const uint64_t* __restrict__ sweep_ptr, int32_t* status, const Rescue rsc,
    const int32_t* __restrict__ rep_slot, const double* __restrict__ ws, int64_t slot_elems,
    int n_waves) {
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + (threadIdx.x >> 6));
    const int hi = __builtin_amdgcn_readfirstlane(rsc.words[3]);
    if (wid == 0 && lane == 0 && hi > 0) atomicAdd(&rsc.words[1], hi);
    const uint64_t sweep = *sweep_ptr;
    for (int i = wid; i < hi; i += n_waves) {
        const DrawTask t = rsc.list[i];
        const ChainInfo& c = chains[t.chain];
        if (c.win_on) continue;  // the windowed kernel draws it (k_backward_win with SLOT)
        const int ro = c.dedup ? row_owner(rsc, c, t.p, t.block) : t.p;
        const int64_t ri = c.blk_off + (int64_t)ro * c.nb + t.block;
        const double* slot = ws + (int64_t)rep_slot[ri] * slot_elems;
        if (ro != t.p && lane == 0) {
            int start, len;
            block_of(c, sweep, t.block, &start, &len);
            const int L_tau = c.L_tau;
            const int qe = start + len >= L_tau ? perm[c.part_off + t.p] : t.p;  // reconnection
            const int e = checked_site(
                paths[c.path_off + (int64_t)((start + len) % L_tau) * c.np + qe], c.N, status,
                t.chain);
            const double hv = slot[(int64_t)(c.B - 1) * c.N + e];
            if (!(hv > 0.0)) set_status(status, FH_ERR_NONFINITE, t.chain);
            blk_logz[c.blk_off + (int64_t)t.p * c.nb + t.block] = blk_la[ri] + log(hv);
        }
        rescue_draws<1>(t, c, tables + tab_g(c), paths, perm, sweep, status, lane, slot);
    }
}

// Shared forward filters, before an FP32 forward pass: one workgroup per (chain, spin, block)
// of the chains with dedup. The rows of a block depend only on the spin's W tables, the block's
// slices and its start site, so every worldline of the (spin, block) is mapped to the lowest
// worldline with the same start site (its representative; itself if it is the lowest); the
// forward kernel runs the representatives only and the backward kernels read their rows.
// For dedup = 1 chains not held this pass it also appends the (spin, block)'s representatives,
// in worldline order and two to a task, to the dense list cpairs (count in words[5]), which the
// split-bf16 forward then takes from the front: its active wavefronts are the first ones
// dispatched, spread over the XCDs, instead of sitting at fixed grid positions that map a whole
// settled batch onto a few compute units. Packed lattices (pack = P) list their representatives
// in prep (count in words[10]) and P^2 of them to a tile in cpack (P = 2: from the front, count
// in words[8]; P = 4: from n_p2 on, count in words[9]).
__global__ __launch_bounds__(kThreads) void k_dedup(const ChainInfo* __restrict__ chains,
                                                    const DrawTask* __restrict__ tasks,
                                                    const int32_t* __restrict__ paths,
                                                    const uint64_t* __restrict__ sweep_ptr,
                                                    int32_t* __restrict__ rep, const Rescue rsc,
                                                    PairTask* __restrict__ cpairs,
                                                    DrawTask* __restrict__ csingles,
                                                    PackTask* __restrict__ cpack, int n_p2,
                                                    int32_t* __restrict__ prep) {
    __shared__ int32_t first[kDedupMaxN];
    __shared__ int32_t rlist[kDedupMaxN];
    __shared__ int32_t n_rep, c_base, p_base;
    const DrawTask t = tasks[blockIdx.x];  // t.p holds the spin
    const ChainInfo& c = chains[t.chain];
    int start, len;
    block_of(c, *sweep_ptr, t.block, &start, &len);
    const int p0 = t.p ? c.n_up : 0, p1 = t.p ? c.np : c.n_up;
    if (c.dedup == 2 && !rescue_held(rsc, t.chain)) {  // shares only in phase A: identity
        for (int q = p0 + threadIdx.x; q < p1; q += blockDim.x)
            rep[c.blk_off + (int64_t)q * c.nb + t.block] = q;
        return;
    }
    for (int i = threadIdx.x; i < c.N; i += blockDim.x) first[i] = 0x7fffffff;
    if (threadIdx.x == 0) n_rep = 0;
    __syncthreads();
    const int32_t* row = paths + c.path_off + (int64_t)start * c.np;
    for (int q = p0 + threadIdx.x; q < p1; q += blockDim.x) {
        const int a = row[q];
        if (a >= 0 && a < c.N) atomicMin(&first[a], q);
    }
    __syncthreads();
    for (int q = p0 + threadIdx.x; q < p1; q += blockDim.x) {
        const int a = row[q];  // an invalid site keeps its own rows (the forward reports it)
        const int r = (a >= 0 && a < c.N) ? first[a] : q;
        rep[c.blk_off + (int64_t)q * c.nb + t.block] = r;
        if (r == q) atomicAdd(&n_rep, 1);
    }
    __syncthreads();
    // the chain's forward recursions in this pass (the FP64 re-filter's phase A sizes by them)
    if (threadIdx.x == 0) atomicAdd(&rsc.words[kRescueChain + 3 * rsc.n_chains + t.chain], n_rep);
    // the 32 x 32 chains' representatives go to cpairs, two to a task; the padded lattices'
    // (16 < L < 32, one worldline to a wavefront) to csingles (count in words[7]); the packed
    // ones to cpack
    const bool pairs = c.L == 32;
    const int PP = c.pack * c.pack;  // worldlines per packed tile
    if (c.dedup != 1 || (pairs ? !cpairs : c.pack ? !cpack : !csingles) ||
        rescue_held(rsc, t.chain))
        return;
    // the representatives in worldline order (first wavefront), then their pairs
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int cnt = 0;
        for (int q0 = p0; q0 < p1; q0 += 64) {
            const int q = q0 + lane;
            bool is_rep = false;
            if (q < p1) {
                const int a = row[q];
                is_rep = !(a >= 0 && a < c.N) || first[a] == q;
            }
            const uint64_t m = __ballot(is_rep);
            if (is_rep) rlist[cnt + __popcll(m & ((1ull << lane) - 1))] = q;
            cnt += __popcll(m);
        }
        if (lane == 0) {
            if (pairs) {
                c_base = atomicAdd(&rsc.words[5], (cnt + 1) / 2);
            } else if (c.pack) {
                p_base = atomicAdd(&rsc.words[10], cnt);
                c_base = atomicAdd(&rsc.words[c.pack == 2 ? 8 : 9], (cnt + PP - 1) / PP) +
                         (c.pack == 2 ? 0 : n_p2);
            } else {
                c_base = atomicAdd(&rsc.words[7], cnt);
            }
        }
    }
    __syncthreads();
    if (c.pack) {
        for (int i = threadIdx.x; i < n_rep; i += blockDim.x) prep[p_base + i] = rlist[i];
        for (int k = threadIdx.x; k * PP < n_rep; k += blockDim.x)
            cpack[c_base + k] = PackTask{t.chain, p_base + k * PP, min(PP, n_rep - k * PP), t.block};
    } else if (pairs) {
        const int npairs = (n_rep + 1) / 2;
        for (int i = threadIdx.x; i < npairs; i += blockDim.x)
            cpairs[c_base + i] = PairTask{t.chain, rlist[2 * i],
                                          2 * i + 1 < n_rep ? rlist[2 * i + 1] : -1, t.block};
    } else {
        for (int i = threadIdx.x; i < n_rep; i += blockDim.x)
            csingles[c_base + i] = DrawTask{t.chain, rlist[i], t.block, 0};
    }
}

// After the FP32 forward pass, one thread per (chain, particle, block) of the chains with dedup:
// a worldline that shares its representative's rows takes the representative's log Z before
// the end weight and reads its own end weight from the representative's end tile
// (C f~ C)(e), exactly what its own recursion would have computed; an end weight below
// kRangeFloor queues the block like the forward kernel's own check.
__global__ void k_member_logz(const ChainInfo* __restrict__ chains, int n_chains,
                              const int32_t* __restrict__ paths, const int32_t* __restrict__ perm,
                              const uint64_t* __restrict__ sweep_ptr,
                              const double* __restrict__ blk_la, const float* __restrict__ endrow,
                              double* __restrict__ blk_logz, int64_t blk_elems, int32_t* status,
                              const Rescue rsc) {
    const uint64_t sweep = *sweep_ptr;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < blk_elems;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int ci = find_chain(n_chains, i, [&](int k) { return chains[k].blk_off; });
        const ChainInfo& c = chains[ci];
        if (c.dedup != 1 || rescue_held(rsc, ci)) continue;
        const int64_t local = i - c.blk_off;
        const int p = (int)(local / c.nb), b = (int)(local % c.nb);
        const int rp = rsc.rep[i];
        if (rp == p) continue;  // a representative: the forward kernel did it
        int start, len;
        block_of(c, sweep, b, &start, &len);
        const int L_tau = c.L_tau;
        const int qe = start + len >= L_tau ? perm[c.part_off + p] : p;  // reconnection
        const int e = checked_site(
            paths[c.path_off + (int64_t)((start + len) % L_tau) * c.np + qe], c.N, status, ci);
        const int64_t ri = c.blk_off + (int64_t)rp * c.nb + b;
        const float hv = endrow[c.end_off + ((int64_t)rp * c.nb + b) * c.N + e];
        if (!(hv >= kRangeFloor)) rescue_push(rsc, c, ci, p, b, kCauseEnd);
        blk_logz[i] = blk_la[ri] + log((double)hv);
    }
}

// Before a forward pass: an empty queue, no block flagged, no chain counted or in phase A (the
// per-chain holds and the redrawn total stay).
__global__ void k_rescue_reset(const Rescue rsc, int64_t n_flags) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i == 0) {
        rsc.words[0] = 0;
        rsc.words[2] = 0;
        rsc.words[3] = 0;
        rsc.words[4] = 0;
        rsc.words[5] = 0;
        rsc.words[6] = 0;
        rsc.words[7] = 0;
        rsc.words[8] = 0;
        rsc.words[9] = 0;
        rsc.words[10] = 0;
    }
    const int n = rsc.n_chains;
    for (int64_t k = i; k < n; k += stride) {
        rsc.words[kRescueChain + k] = 0;
        rsc.words[kRescueChain + 2 * n + k] = 0;
        rsc.words[kRescueChain + 3 * n + k] = 0;
        // the hold: a chain that entered the previous pass in FP32 and left it held failed its
        // retry (or first met a floor): hold it for the current length, and double that for
        // the next failure; a pass in FP32 that queued nothing resets the length
        int hold = rsc.words[kRescueChain + n + k];
        const int hold0 = rsc.words[kRescueChain + 4 * n + k];
        int len = max(rsc.words[kRescueChain + 5 * n + k], kRescueHold);
        if (hold0 == 0 && hold > 0) {
            hold = len;
            len = min(2 * len, kRescueHoldMax);
        } else if (hold0 == 0) {
            len = kRescueHold;
        }
        rsc.words[kRescueChain + n + k] = hold;
        rsc.words[kRescueChain + 4 * n + k] = hold;
        rsc.words[kRescueChain + 5 * n + k] = len;
    }
    for (int64_t k = i; k < n_flags; k += stride) rsc.flags[k] = 0;
}

// After k_rescue_reset and k_dedup, before a sweep's FP32 forward pass, one workgroup: every
// block of each chain held on the FP64 re-filter (fp64_circulant) is queued, in chain order, as
// phase A, and the chain is marked, while the running total of the held chains' forward
// recursions (their representatives) fits the n_slots slots; the FP32 kernels skip held chains
// and phase A re-filters them beside the FP32 passes (a held chain left out is queued whole after
// the forward pass, for phase 2). The queue is empty before this kernel, so the entries are laid
// down in place. Phase A also gets the dense list of its representatives, arep.
__global__ __launch_bounds__(kThreads) void k_rescue_held(const ChainInfo* __restrict__ chains,
                                                          const Rescue rsc, int n_slots,
                                                          int shared, DrawTask* __restrict__ arep) {
    // one thread per chain, kThreads chains at a time: block-wide inclusive scans of the held
    // chains' recursions (admission: the running total fits the slots) and of the admitted
    // chains' blocks (their place in the queue)
    __shared__ int scan_rec[kThreads], scan_blk[kThreads], adm_share[kThreads];
    const int tid = threadIdx.x, n = rsc.n_chains;
    int off = 0, slots = 0;
    for (int c0 = 0; c0 < n; c0 += kThreads) {
        const int ci = c0 + tid;
        bool held = false;
        int nblk = 0, nrec = 0;
        bool share = false;
        if (ci < n) {
            const ChainInfo& c = chains[ci];
            held = fp64_circulant(c.L) && rescue_held(rsc, ci);
            nblk = c.np * c.nb;
            share = shared && c.dedup;
            nrec = held ? (share ? rsc.words[kRescueChain + 3 * n + ci] : nblk) : 0;
        }
        scan_rec[tid] = nrec;
        __syncthreads();
        for (int d = 1; d < kThreads; d <<= 1) {  // inclusive scan of the recursions
            const int v = tid >= d ? scan_rec[tid - d] : 0;
            __syncthreads();
            scan_rec[tid] += v;
            __syncthreads();
        }
        const bool admit = held && slots + scan_rec[tid] <= n_slots;
        scan_blk[tid] = admit ? nblk : 0;
        adm_share[tid] = admit ? (share ? 2 : 1) : 0;
        __syncthreads();
        for (int d = 1; d < kThreads; d <<= 1) {  // inclusive scan of the admitted blocks
            const int v = tid >= d ? scan_blk[tid - d] : 0;
            __syncthreads();
            scan_blk[tid] += v;
            __syncthreads();
        }
        if (admit) rsc.words[kRescueChain + 2 * n + ci] = 1;
        // the admitted chains' blocks, one chain after another, by the whole workgroup
        for (int k = 0; k < kThreads && c0 + k < n; ++k) {
            if (!adm_share[k]) continue;
            const int ck = c0 + k;
            const ChainInfo& c = chains[ck];
            const int nb_k = c.np * c.nb, base = off + scan_blk[k] - nb_k;
            for (int i = tid; i < nb_k; i += kThreads) {  // i = p nb + block
                rsc.flags[c.blk_off + i] = 1;
                rsc.list[base + i] = DrawTask{ck, i / c.nb, i % c.nb, 0};
                // the representatives, in no particular order (at most n_slots of them)
                if (adm_share[k] == 1 || rsc.rep[c.blk_off + i] == i / c.nb)
                    arep[atomicAdd(&rsc.words[6], 1)] = DrawTask{ck, i / c.nb, i % c.nb, 0};
            }
        }
        // the chunk's admitted recursions: the admitted chains are the held ones up to the last
        // admitted, whose inclusive scan is their total
        __shared__ int adm_rec;
        if (tid == 0) adm_rec = 0;
        __syncthreads();
        if (admit) atomicMax(&adm_rec, scan_rec[tid]);
        __syncthreads();
        slots += adm_rec;
        off += scan_blk[kThreads - 1];
        __syncthreads();  // the scans' storage and adm_rec are reused by the next chunk
    }
    if (tid == 0) {
        rsc.words[0] = off;
        rsc.words[3] = off;
    }
}

// After the FP32 forward pass, one workgroup per chain: a chain with more than whole_min blocks
// queued in this pass, or still held from an earlier such pass, has all its blocks queued for the
// FP64 re-filter; its hold then counts down (k_rescue_reset sets its length at the next pass).
__global__ __launch_bounds__(kThreads) void k_rescue_expand(const ChainInfo* __restrict__ chains,
                                                            const Rescue rsc) {
    const int ci = blockIdx.x;
    const ChainInfo& c = chains[ci];
    const int cnt = rsc.words[kRescueChain + ci];
    const int hold = rsc.words[kRescueChain + rsc.n_chains + ci];
    const bool many = cnt > c.whole_min;
    const bool whole = many || hold > 0;
    if (whole)
        for (int i = threadIdx.x; i < c.np * c.nb; i += blockDim.x)
            rescue_enqueue(rsc, c, ci, i / c.nb, i % c.nb);
    __syncthreads();  // every thread read the count and the hold before they change
    if (threadIdx.x == 0) {
        rsc.words[kRescueChain + rsc.n_chains + ci] = many ? kRescueHold : max(hold - 1, 0);
        if (whole) {
            atomicAdd(&rsc.words[2], 1);
            rsc.words[kRescueChain + ci] = cnt + c.np * c.nb;  // the chain has queued blocks
        }
    }
}

// Before the FP64 re-filter, one workgroup per (chain, slice) of the chains with blocks in the
// phase's part of the queue (phase 0: queued; 1: in phase A; 2: queued, not in phase A):
// W~ = exp(coef aux - m) in FP64 for both spins (the FP32 tables may hold zeros), with the
// shift m of the FP32 tables.
__global__ __launch_bounds__(kThreads) void k_rescue_potentials(
    const ChainInfo* __restrict__ chains, int n_chains, const float* __restrict__ aux,
    const double* __restrict__ wshift, double* __restrict__ W64, int64_t aux_elems,
    int64_t total_slices, const Rescue rsc, int phase) {
    const int gs = blockIdx.x;
    const int ci = find_chain(n_chains, gs, [&](int i) { return chains[i].slice_off; });
    const bool in_a = rsc.words[kRescueChain + 2 * n_chains + ci] != 0;
    const bool queued = phase == 1 ? in_a
                                   : rsc.words[kRescueChain + ci] != 0 && !(phase == 2 && in_a);
    if (!queued) return;  // nothing of this chain is in this phase
    const ChainInfo& c = chains[ci];
    const int64_t base = c.aux_off + (int64_t)(gs - c.slice_off) * c.N;
    const double mu = wshift[gs], md = wshift[total_slices + gs];
    for (int r = threadIdx.x; r < c.N; r += blockDim.x) {
        const double v = (double)aux[base + r];
        W64[base + r] = exp(c.coef_up * v - mu);
        W64[aux_elems + base + r] = exp(c.coef_dn * v - md);
    }
}

// After the backward pass of a sweep: moves the plan's windowed chains between the windowed
// kernel and the full-row kernels (the draws are the same either way). When the first window
// left more than 3/20 of the windowed chains' draws uncertified, the windowed kernel runs slower
// than the full-row one (its four worldlines per wavefront wait for every fallback), and the
// next `hold` backward passes use the full-row kernels; then the window is tried again. hold
// starts at 16 and doubles, up to 64, while the retries keep failing. The switch is plan-wide:
// both kernels are latency-bound, so splitting the chains between them would cost the sum of
// their times. One workgroup; the per-chain counts are summed in chain order.
__global__ void k_bw_adapt(const ChainInfo* __restrict__ chains, int n_chains,
                           int32_t* __restrict__ bw_state) {
    __shared__ int64_t part[2][kThreads];
    int64_t unc = 0, draws = 0;
    for (int ci = threadIdx.x; ci < n_chains; ci += blockDim.x) {
        const ChainInfo& c = chains[ci];
        if (!c.win_on) continue;
        unc += bw_state[kBwCounts + ci];
        draws += (int64_t)c.np * (c.L_tau - c.nb);
        bw_state[kBwCounts + ci] = 0;
    }
    part[0][threadIdx.x] = unc;
    part[1][threadIdx.x] = draws;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 1; k < (int)blockDim.x; ++k) {
        unc += part[0][k];
        draws += part[1][k];
    }
    if (bw_state[0] > 0) {  // a full-row pass just ran
        bw_state[0] -= 1;
    } else if (unc * 20 > draws * 3) {
        bw_state[1] = bw_state[1] == 0 ? 16 : min(2 * bw_state[1], 64);
        bw_state[0] = bw_state[1];
    } else {
        bw_state[1] = 0;
    }
}

// One wavefront per (chain, worldline, block) of the chains with L != 32, the body chosen per
// chain: up to 4 sites per lane (N <= 256), or up to 16 (N <= 1024).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_backward_fast(
    const ChainInfo* __restrict__ chains, const DrawTask* __restrict__ tasks, int n_tasks,
    const double* __restrict__ tables, const T* __restrict__ filt, int32_t* __restrict__ paths, const int32_t* __restrict__ perm,
    const uint64_t* __restrict__ sweep_ptr, int32_t* status, const int32_t* __restrict__ bw_state,
    const Rescue rsc) {
    __shared__ double gsh[kWaves][kMaxL];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int task = blockIdx.x * kWaves + wv;
    const bool active = task < n_tasks && !on_window(chains, tasks[task].chain, bw_state);
    DrawTask t = {0, 0, 0, 0};
    if (active) {
        t = tasks[task];
        const ChainInfo& c0 = chains[t.chain];
        for (int m = lane; m < c0.L; m += 64) gsh[wv][m] = tables[tab_g(c0) + m];
    }
    __syncthreads();  // the only barrier; every wave reaches it
    if (!active) return;
    const ChainInfo& c = chains[t.chain];
    const uint64_t sweep = *sweep_ptr;
    if (c.N <= 256)
        backward_task<T, false, 0, 4>(t, c, gsh[wv], filt, paths, perm, sweep, status, lane,
                                      rsc);
    else
        backward_task<T, false, 0, 16>(t, c, gsh[wv], filt, paths, perm, sweep, status, lane,
                                       rsc);
}


// Local link updates (Sec. 3.5.1, eq. Rlocal, site form). A move proposes to take the site r of
// slice l of a worldline to a nearest neighbour r' (top two bits of Philox word x1: +x, -x, +y,
// -y; periodic) with the sites r_prev, r_next of the two adjacent slices fixed, and is taken iff
// u < R with
//   R = exp(coef (aux_l(r') - aux_l(r))) G(r' - r_prev) G(r_next - r') / [G(r - r_prev) G(r_next - r)],
// G(d) = g(d_x) g(d_y), everything in FP64 (W_l(r')/W_l(r) written through the field). Counter
// (particle, slice, sweep, kTagLocal + 256 pass); u from word x0.
template <typename T>
__device__ inline int local_move(const ChainInfo& c, const double* g, const T* ax, int l, int cur,
                                 int prev, int next, double coef, int p, uint64_t sweep, int ps) {
    const int L = c.L;
    auto G = [&](int a, int b) {  // G(a - b) on the periodic lattice
        int dx = a % L - b % L;
        dx += dx < 0 ? L : 0;
        int dy = a / L - b / L;
        dy += dy < 0 ? L : 0;
        return g[dx] * g[dy];
    };
    const u64x4 w = philox4x64_10((uint64_t)p, (uint64_t)l, sweep,
                                  kTagLocal + 256ull * (uint64_t)ps, c.seed, 0);
    const int e = (int)(w.x1 >> 62);
    const double u = u01_from(w.x0);
    const int x = cur % L, y = cur / L;
    const int nx = e == 0 ? (x + 1 == L ? 0 : x + 1) : e == 1 ? (x == 0 ? L - 1 : x - 1) : x;
    const int ny = e == 2 ? (y + 1 == L ? 0 : y + 1) : e == 3 ? (y == 0 ? L - 1 : y - 1) : y;
    const int cand = nx + L * ny;
    const double dA = (double)ax[(int64_t)l * c.N + cand] - (double)ax[(int64_t)l * c.N + cur];
    const double R =
        exp(coef * dA) * ((G(cand, prev) * G(next, cand)) / (G(cur, prev) * G(next, cur)));
    return u < R ? cand : cur;
}

// One pass of local updates: a checkerboard in tau, four launches. PHASE 0 moves the odd
// interior slices 1, 3, ... <= L_tau-2 of every worldline, PHASE 1 the even interior slices
// 2, 4, ... <= L_tau-2, PHASE 2 slice 0 (whose previous slice is slice L_tau-1 of perm_inv[p]),
// PHASE 3 slice L_tau-1 (whose next slice is slice 0 of perm[p]). A move sees only the two
// adjacent slices, which belong to other phases, so the moves of a launch are independent: one
// thread per (worldline, slice). Interior phases take k0 plus the grid's y index as the slice
// pair k (slice 2k + 1 or 2k + 2); threads past a chain's last slice of the phase leave.
template <typename T, int PHASE>
__global__ __launch_bounds__(kThreads) void k_local(const ChainInfo* __restrict__ chains,
                                                    int n_chains, int64_t particles,
                                                    const double* __restrict__ tables,
                                                    const T* __restrict__ aux,
                                                    int32_t* __restrict__ paths,
                                                    const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ perm_inv,
                                                    const uint64_t* __restrict__ sweep_ptr,
                                                    int ps, int k0, int32_t* status) {
    const int64_t gp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gp >= particles) return;
    const int ci = find_chain(n_chains, gp, [&](int i) { return chains[i].part_off; });
    const ChainInfo& c = chains[ci];
    const int p = (int)(gp - c.part_off);
    const int N = c.N, L_tau = c.L_tau;
    const int64_t np = c.np;
    int l, qprev = p, qnext = p;  // slice, and the worldlines holding its neighbours
    if (PHASE < 2) {
        l = 2 * (k0 + (int)blockIdx.y) + 1 + PHASE;
        if (l > L_tau - 2) return;
    } else if (PHASE == 2) {
        l = 0;
        qprev = perm_inv[c.part_off + p];
    } else {
        l = L_tau - 1;
        qnext = perm[c.part_off + p];
    }
    const double* g = tables + tab_g(c);
    const double coef = p >= c.n_up ? c.coef_dn : c.coef_up;
    const T* ax = aux + c.aux_off;
    int32_t* col = paths + c.path_off;  // slice l of worldline q at col[l * np + q]
    const uint64_t sweep = *sweep_ptr;
    const int lp = l == 0 ? L_tau - 1 : l - 1, ln = l == L_tau - 1 ? 0 : l + 1;
    const int prev = col[(int64_t)lp * np + qprev];
    const int next = col[(int64_t)ln * np + qnext];
    const int cur = col[(int64_t)l * np + p];
    if (prev < 0 || prev >= N || next < 0 || next >= N || cur < 0 || cur >= N) {
        set_status(status, FH_ERR_BAD_PATH, ci);
        return;
    }
    const int taken = local_move(c, g, ax, l, cur, prev, next, coef, p, sweep, ps);
    if (taken != cur) col[(int64_t)l * np + p] = taken;
}

// Pair swaps of the reconnections at tau = beta (Sec. 3.5.6), one thread per worldline; the
// first worldline p of each candidate pair of pass ps, (p0 + o + 2i, p0 + o + 2i + 1) within its
// spin, o = ps mod 2, trades perm[p] and perm[q = p + 1] iff u < R,
//   R = G(r^{P(q)}_0 - r^p_{L-1}) G(r^{P(p)}_0 - r^q_{L-1}) / [G(r^{P(p)}_0 - r^p_{L-1}) G(r^{P(q)}_0 - r^q_{L-1})]
// (only the two boundary hops change), u from Philox (p, 0, sweep, kTagPerm + 256 ps). An accepted
// swap flips the chain's sign (+1 <-> -1 by one atomic xor). The pairs of a pass are disjoint.
__global__ __launch_bounds__(kThreads) void k_perm_update(
    const ChainInfo* __restrict__ chains, int n_chains, int64_t particles,
    const double* __restrict__ tables, const int32_t* __restrict__ paths, int32_t* perm,
    int32_t* perm_inv, int32_t* sign, const uint64_t* __restrict__ sweep_ptr, int ps,
    int32_t* status) {
    const int64_t gp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gp >= particles) return;
    const int ci = find_chain(n_chains, gp, [&](int i) { return chains[i].part_off; });
    const ChainInfo& c = chains[ci];
    const int p = (int)(gp - c.part_off);
    const int p0 = p < c.n_up ? 0 : c.n_up, n = p < c.n_up ? c.n_up : c.n_dn;
    const int k = p - p0 - (ps & 1);
    if (k < 0 || (k & 1) || p + 1 >= p0 + n) return;
    const int q = p + 1, L = c.L, N = c.N;
    const double* g = tables + tab_g(c);
    auto G = [&](int a, int b) {
        int dx = a % L - b % L;
        dx += dx < 0 ? L : 0;
        int dy = a / L - b / L;
        dy += dy < 0 ? L : 0;
        return g[dx] * g[dy];
    };
    const int32_t* col = paths + c.path_off;
    const int64_t last = (int64_t)(c.L_tau - 1) * c.np;
    const int Pp = perm[c.part_off + p], Pq = perm[c.part_off + q];
    const int lp = col[last + p], lq = col[last + q], fp = col[Pp], fq = col[Pq];
    if (lp < 0 || lp >= N || lq < 0 || lq >= N || fp < 0 || fp >= N || fq < 0 || fq >= N) {
        set_status(status, FH_ERR_BAD_PATH, ci);
        return;
    }
    const double R = (G(fq, lp) * G(fp, lq)) / (G(fp, lp) * G(fq, lq));
    const u64x4 w = philox4x64_10((uint64_t)p, 0, *sweep_ptr, kTagPerm + 256ull * (uint64_t)ps,
                                  c.seed, 0);
    if (u01_from(w.x0) < R) {
        perm[c.part_off + p] = Pq;
        perm[c.part_off + q] = Pp;
        perm_inv[c.part_off + Pq] = p;
        perm_inv[c.part_off + Pp] = q;
        atomicXor(&sign[ci], (int32_t)0xFFFFFFFE);
    }
}

// Occupation counts of one slice (LDS histogram) and the exact field draw of every site:
// Ising: s = +1 iff u < (1 + tanh(lambda (n_up - n_dn))) / 2; Gaussian: sigma = a (n - 1/2) + z.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gibbs(const ChainInfo* __restrict__ chains,
                                                    int n_chains, const int32_t* __restrict__ paths,
                                                    T* __restrict__ aux,
                                                    const uint64_t* __restrict__ sweep_ptr,
                                                    int32_t* status, int maxN) {
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t* cnt = (int32_t*)smem;  // [2][maxN]
    const int gs = blockIdx.x;
    const int ci = find_chain(n_chains, gs, [&](int i) { return chains[i].slice_off; });
    const ChainInfo& c = chains[ci];
    const int l = (int)(gs - c.slice_off);
    const uint64_t sweep = *sweep_ptr;
    for (int r = threadIdx.x; r < 2 * c.N; r += blockDim.x) cnt[(r / c.N) * maxN + r % c.N] = 0;
    __syncthreads();
    const int32_t* pl = paths + c.path_off + (int64_t)l * c.np;
    for (int p = threadIdx.x; p < c.np; p += blockDim.x) {
        const int r = pl[p];
        if (r >= 0 && r < c.N)
            atomicAdd(&cnt[(p >= c.n_up ? maxN : 0) + r], 1);
        else
            set_status(status, FH_ERR_BAD_PATH, ci);
    }
    __syncthreads();
    T* al = aux + c.aux_off + (int64_t)l * c.N;
    for (int r = threadIdx.x; r < c.N; r += blockDim.x) {
        const int nu = cnt[r], nd = cnt[maxN + r];
        const u64x4 x = philox4x64_10((uint64_t)r, (uint64_t)l, sweep, kTagGibbs, c.seed, 0);
        double v;
        if (c.hs_kind == FH_HS_GAUSS) {
            v = c.gauss_a * ((double)(nu + nd) - 0.5) + normal_from(x.x0, x.x1);
        } else {
            const double pp = (1.0 + tanh(c.hirsch_lambda * (double)(nu - nd))) / 2.0;
            v = u01_from(x.x0) < pp ? 1.0 : -1.0;
        }
        al[r] = (T)v;
    }
}

// Langevin proposal for the Gaussian field (MALA), one thread per field value:
//   sigma' = sigma + h (-sigma - a/2 + dlogZ(sigma)) + eps xi,  h = eps^2 / 2,
// xi from the Philox counter (site, slice, sweep, kTagMala) by Box-Muller. Ising-field chains
// copy their field (they are never accepted).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mala_propose(
    const ChainInfo* __restrict__ chains, int n_chains, int64_t aux_elems,
    const T* __restrict__ aux, const T* __restrict__ dlogz, T* __restrict__ prop, double eps,
    const uint64_t* __restrict__ sweep_ptr) {
    const uint64_t sweep = *sweep_ptr;
    const double h = 0.5 * eps * eps;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < aux_elems;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int ci = find_chain(n_chains, e, [&](int i) { return chains[i].aux_off; });
        const ChainInfo& c = chains[ci];
        const double s = (double)aux[e];
        if (c.hs_kind != FH_HS_GAUSS) {
            prop[e] = aux[e];
            continue;
        }
        const int64_t off = e - c.aux_off;
        const int l = (int)(off / c.N), r = (int)(off % c.N);
        const u64x4 x = philox4x64_10((uint64_t)r, (uint64_t)l, sweep, kTagMala, c.seed, 0);
        const double g = -s - 0.5 * c.gauss_a + (double)dlogz[e];
        prop[e] = (T)(s + h * g + eps * normal_from(x.x0, x.x1));
    }
}

// MALA acceptance, one workgroup per chain: the Metropolis-Hastings ratio of the Langevin move
//   log alpha = [prior + log Z_path](sigma') - [prior + log Z_path](sigma)
//               - |sigma - sigma' - h g(sigma')|^2 / (2 eps^2) + |sigma' - sigma - h g(sigma)|^2 / (2 eps^2),
// prior = sum (-sigma^2/2 - a sigma/2), g = -sigma - a/2 + dlogZ, summed in FP64 in a fixed
// order; u from Philox (0, 0, sweep, kTagMalaAccept); the chain's field becomes sigma' iff
// u < exp(min(log alpha, 0)). accepted[c] = 1 / 0, -1 for Ising-field chains.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mala_accept(
    const ChainInfo* __restrict__ chains, T* __restrict__ aux, const T* __restrict__ prop,
    const T* __restrict__ g0, const T* __restrict__ g1, const double* __restrict__ logz0,
    const double* __restrict__ logz1, double eps, const uint64_t* __restrict__ sweep_ptr,
    int32_t* __restrict__ accepted) {
    __shared__ double red[3][kThreads];
    __shared__ int take;
    const ChainInfo& c = chains[blockIdx.x];
    if (c.hs_kind != FH_HS_GAUSS) {
        if (threadIdx.x == 0 && accepted) accepted[blockIdx.x] = -1;
        return;  // whole workgroup; no barrier reached
    }
    const double h = 0.5 * eps * eps, a = c.gauss_a;
    const int64_t n = (int64_t)c.L_tau * c.N;
    double lp = 0.0, fwd = 0.0, rev = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t e = c.aux_off + i;
        const double s = (double)aux[e], sp = (double)prop[e];
        const double gs = -s - 0.5 * a + (double)g0[e], gp = -sp - 0.5 * a + (double)g1[e];
        lp += (-0.5 * sp * sp - 0.5 * a * sp) - (-0.5 * s * s - 0.5 * a * s);
        const double df = sp - s - h * gs, dr = s - sp - h * gp;
        fwd += df * df;
        rev += dr * dr;
    }
    red[0][threadIdx.x] = lp;
    red[1][threadIdx.x] = fwd;
    red[2][threadIdx.x] = rev;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double la = red[0][0] + logz1[blockIdx.x] - logz0[blockIdx.x] -
                          red[2][0] / (2.0 * eps * eps) + red[1][0] / (2.0 * eps * eps);
        const u64x4 x = philox4x64_10(0, 0, *sweep_ptr, kTagMalaAccept, c.seed, 0);
        take = u01_from(x.x0) < exp(la < 0.0 ? la : 0.0) ? 1 : 0;
        if (accepted) accepted[blockIdx.x] = take;
    }
    __syncthreads();
    if (take)
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) aux[c.aux_off + i] = prop[c.aux_off + i];
}

// Equal-time observables of one slice (Sec. 4), one workgroup per (chain, slice): occupation
// counts by an LDS histogram, S^z = (n_up - n_dn) / 2, F = 2D FFT of S^z (the Stockham stages of
// the forward filter, FP64), S(k) = |F(k)|^2 / N and, from the unscaled inverse FFT of |F|^2,
// C(r) = (1/N) sum_j S^z_{j+r} S^z_j = IFFT(|F|^2)(r) / N^2. Rows go to the slice's place in
// sk / cr (packed like aux); the site sums of n_up n_dn and (n_up - n_dn)^2 to sums[slice][2].
__global__ __launch_bounds__(kThreads) void k_measure(const ChainInfo* __restrict__ chains,
                                                      int n_chains, const double* __restrict__ tables,
                                                      const int32_t* __restrict__ paths,
                                                      double* __restrict__ sk, double* __restrict__ cr,
                                                      double* __restrict__ sums, int32_t* status,
                                                      int maxN, int maxL) {
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<double>* A = (cpx<double>*)smem;  // [maxN]
    cpx<double>* S = A + maxN;            // [maxN] FFT scratch; the histogram lives here first
    cpx<double>* tw = S + maxN;           // [maxL]
    double* red = (double*)(tw + maxL);   // [2][kWaves]
    int32_t* cnt = (int32_t*)S;           // [2][maxN] ints fit in S (16 bytes per element)
    const int64_t gs = blockIdx.x;
    const int ci = find_chain(n_chains, gs, [&](int i) { return chains[i].slice_off; });
    const ChainInfo& c = chains[ci];
    const int l = (int)(gs - c.slice_off);
    const int N = c.N, L = c.L;
    for (int r = threadIdx.x; r < 2 * N; r += blockDim.x) cnt[r] = 0;
    const double* twt = tables + tab_tw(c);
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = {twt[2 * m], twt[2 * m + 1]};
    __syncthreads();
    const int32_t* pl = paths + c.path_off + (int64_t)l * c.np;
    for (int p = threadIdx.x; p < c.np; p += blockDim.x) {
        const int r = pl[p];
        if (r >= 0 && r < N)
            atomicAdd(&cnt[(p >= c.n_up ? N : 0) + r], 1);
        else
            set_status(status, FH_ERR_BAD_PATH, ci);
    }
    __syncthreads();
    double d = 0.0, m2 = 0.0;
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        const int nu = cnt[r], nd = cnt[N + r];
        A[r] = {0.5 * (double)(nu - nd), 0.0};
        d += (double)nu * (double)nd;
        m2 += (double)(nu - nd) * (double)(nu - nd);
    }
    d = wave_sum(d);
    m2 = wave_sum(m2);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[wv] = d;
        red[kWaves + wv] = m2;
    }
    __syncthreads();  // also: the histogram in S is read before the FFT reuses S
    if (threadIdx.x == 0) {
        double sd = 0.0, sm = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            sd += red[w];
            sm += red[kWaves + w];
        }
        sums[2 * gs] = sd;
        sums[2 * gs + 1] = sm;
    }
    fft2d<double, false>(A, S, L, c.plan, tw);
    double* skr = sk + c.aux_off + (int64_t)l * N;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const double p2 = A[k].re * A[k].re + A[k].im * A[k].im;
        skr[k] = p2 / (double)N;
        A[k] = {p2, 0.0};
    }
    __syncthreads();
    fft2d<double, true>(A, S, L, c.plan, tw);
    double* crr = cr + c.aux_off + (int64_t)l * N;
    const double inv = 1.0 / ((double)N * (double)N);
    for (int r = threadIdx.x; r < N; r += blockDim.x) crr[r] = A[r].re * inv;
}

// Slice averages of k_measure's rows, summed in slice order: S(k), C(r) per site of every chain
// (threads 0 .. total_sites-1), then D and the local moment per chain.
__global__ __launch_bounds__(kThreads) void k_measure_reduce(
    const ChainInfo* __restrict__ chains, int n_chains, int64_t total_sites,
    const double* __restrict__ sk, const double* __restrict__ cr, const double* __restrict__ sums,
    double* __restrict__ Sk, double* __restrict__ Cr, double* __restrict__ D,
    double* __restrict__ S2) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < total_sites) {
        const int ci = find_chain(n_chains, t, [&](int i) { return chains[i].site_off; });
        const ChainInfo& c = chains[ci];
        const int k = (int)(t - c.site_off);
        double a = 0.0, b = 0.0;
        for (int l = 0; l < c.L_tau; ++l) {
            a += sk[c.aux_off + (int64_t)l * c.N + k];
            b += cr[c.aux_off + (int64_t)l * c.N + k];
        }
        if (Sk) Sk[t] = a / c.L_tau;
        if (Cr) Cr[t] = b / c.L_tau;
    } else if (t < total_sites + n_chains) {
        const ChainInfo& c = chains[t - total_sites];
        double a = 0.0, b = 0.0;
        for (int l = 0; l < c.L_tau; ++l) {
            a += sums[2 * (c.slice_off + l)];
            b += sums[2 * (c.slice_off + l) + 1];
        }
        const double n = (double)c.L_tau * (double)c.N;
        if (D) D[t - total_sites] = a / n;
        if (S2) S2[t - total_sites] = 0.75 * b / n;
    }
}

// Adjoint of the forward filter over the ring anchored at `anchor` (one block of length L_tau,
// closing on the anchor site e of the reconnected worldline, e = a without reconnection):
// forward pass storing f~_j (j = 0..L_tau-1), then backward messages
//   u_{L_tau} = delta_e;  beta_j = G * u_{j+1};  u_j = W_j . beta_j / sum   (FFT convolution)
// with d log Z / d log W_j(r) = f~_j(r) beta_j(r) / <f~_j, beta_j> accumulated into grad_aux
// (times the spin's coefficient) and d log Z / dt += <dG/dt * u_{j+1}, f~_j> / <beta_j, f~_j>.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_grad(
    const ChainInfo* __restrict__ chains, const GroupTask* __restrict__ groups,
    const double* __restrict__ tables, const T* __restrict__ aux, const T* __restrict__ W,
    const double* __restrict__ wshift, int64_t aux_elems, int64_t total_slices,
    const int32_t* __restrict__ paths, T* __restrict__ filt, double* __restrict__ blk_logz,
    double* __restrict__ dt_out, T* __restrict__ gpart, int anchor,
    const int32_t* __restrict__ perm, int32_t* status, int maxN, int maxL) {
    extern __shared__ __align__(16) unsigned char smem[];
    FftLds<T> l = carve<T>(smem, maxN, maxL, true);
    const GroupTask g = groups[blockIdx.x];  // one or two worldlines of one (chain, spin)
    const PairTask t = {g.chain, g.p0, g.count > 1 ? g.p0 + 1 : -1, 0};
    const ChainInfo& c = chains[t.chain];
    const int N = c.N, L = c.L, L_tau = c.L_tau;
    const bool has_b = t.p_b >= 0;
    const int spin = t.p_a >= c.n_up ? 1 : 0;
    const double coef = spin ? c.coef_dn : c.coef_up;
    const T* Wsp = W + spin * aux_elems + c.aux_off;
    const double* shift = wshift + spin * total_slices + c.slice_off;
    const int32_t* pc = paths + c.path_off;
    const int a_a = checked_site(pc[(int64_t)anchor * c.np + t.p_a], N, status, t.chain);
    const int a_b = has_b ? checked_site(pc[(int64_t)anchor * c.np + t.p_b], N, status, t.chain) : 0;
    // the ring closes on the anchor site of the reconnected worldline (itself for the identity)
    const int e_a = checked_site(pc[(int64_t)anchor * c.np + perm[c.part_off + t.p_a]], N, status,
                                 t.chain);
    const int e_b = has_b ? checked_site(pc[(int64_t)anchor * c.np + perm[c.part_off + t.p_b]], N,
                                         status, t.chain)
                          : 0;
    load_chain_tables(c, tables, l);
    T* row_a = filt + c.filt_off + (int64_t)t.p_a * L_tau * N;
    T* row_b = has_b ? filt + c.filt_off + (int64_t)t.p_b * L_tau * N : nullptr;
    double lza, lzb;
    forward_pass<T>(c, tables, Wsp, shift, aux + c.aux_off, coef, anchor, L_tau, a_a, e_a, a_b,
                    e_b, has_b, row_a, row_b, 0, l, &lza, &lzb, status, t.chain);
    const double* gh = tables + tab_ghat(c);
    const double* dgh = tables + tab_dghat(c);
    for (int r = threadIdx.x; r < N; r += blockDim.x)
        l.U[r] = {r == e_a ? T(1) : T(0), (has_b && r == e_b) ? T(1) : T(0)};
    double dta = 0.0, dtb = 0.0;
    // the pair's own partial field-gradient slab [L_tau][N]; k_gpart_reduce adds a chain's slabs
    // in group order, so the field gradient is the same on every call
    T* gl = gpart ? gpart + g.part_off : nullptr;
    for (int j = L_tau - 1; j >= 0; --j) {
        const int lj = (anchor + j) % L_tau;
        __syncthreads();
        fft2d<T, false>(l.U, l.S, L, c.plan, l.tw);
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            const cpx<T> s = l.U[k];
            const T m = (T)gh[k], dm = (T)dgh[k];
            l.A[k] = {s.re * m, s.im * m};
            l.U[k] = {s.re * dm, s.im * dm};
        }
        __syncthreads();
        fft2d<T, true>(l.A, l.S, L, c.plan, l.tw);   // beta_j = G * u_{j+1}
        fft2d<T, true>(l.U, l.S, L, c.plan, l.tw);   // dG/dt * u_{j+1}
        const T* fa = row_a + (int64_t)j * N;
        const T* fb = has_b ? row_b + (int64_t)j * N : nullptr;
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r = threadIdx.x; r < N; r += blockDim.x) {
            const double va = (double)fa[r];
            s[0] += (double)l.U[r].re * va;
            s[1] += (double)l.A[r].re * va;
            if (has_b) {
                const double vb = (double)fb[r];
                s[2] += (double)l.U[r].im * vb;
                s[3] += (double)l.A[r].im * vb;
            }
        }
        block_sum<4>(s, l.red);
        dta += s[0] / s[1];
        if (has_b) dtb += s[2] / s[3];
        if (gl) {
            const double ka = coef / s[1], kb = has_b ? coef / s[3] : 0.0;
            for (int r = threadIdx.x; r < N; r += blockDim.x) {
                double v = ka * (double)fa[r] * (double)l.A[r].re;
                if (has_b) v += kb * (double)fb[r] * (double)l.A[r].im;
                gl[(int64_t)lj * N + r] = (T)v;
            }
        }
        if (j > 0) {
            const T* Wl = Wsp + (int64_t)lj * N;
            double z[2] = {0.0, 0.0};
            for (int r = threadIdx.x; r < N; r += blockDim.x) {
                const T w = Wl[r];
                const cpx<T> v = {l.A[r].re * w, l.A[r].im * w};
                l.U[r] = v;
                z[0] += (double)v.re;
                z[1] += (double)v.im;
            }
            block_sum<2>(z, l.red);
            if (!(z[0] > 0.0) || !isfinite(z[0]))
                if (threadIdx.x == 0) set_status(status, FH_ERR_NONFINITE, t.chain);
            const T ia = (T)(1.0 / z[0]), ib = has_b ? (T)(1.0 / z[1]) : T(0);
            for (int r = threadIdx.x; r < N; r += blockDim.x) {
                l.U[r].re *= ia;
                l.U[r].im *= ib;
            }
        }
    }
    if (threadIdx.x == 0) {
        blk_logz[c.blk_off + (int64_t)t.p_a * c.nb] = lza;
        dt_out[c.part_off + t.p_a] = dta;
        if (has_b) {
            blk_logz[c.blk_off + (int64_t)t.p_b * c.nb] = lzb;
            dt_out[c.part_off + t.p_b] = dtb;
        }
    }
}

// Per chain, in particle order: logZ = sum of ring log Z_p, grad_t = sum of d log Z_p / dt.
// Per chain: log Z_path = sum of the ring log Z of its worldlines, d/dt = sum of theirs. One
// wavefront per chain; lane k sums worldlines k, k + 64, ... in order, then a fixed butterfly adds
// the lanes, so the result is the same on every call.
__global__ void k_grad_reduce(const ChainInfo* __restrict__ chains, int n_chains,
                              const double* __restrict__ blk_logz, const double* __restrict__ dt,
                              double* logZ, double* grad_t) {
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= n_chains) return;
    const ChainInfo& ci = chains[c];
    double a = 0.0, b = 0.0;
    for (int p = lane; p < ci.np; p += 64) {
        a += blk_logz[ci.blk_off + (int64_t)p * ci.nb];
        b += dt[ci.part_off + p];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) {
        if (logZ) logZ[c] = a;
        if (grad_t) grad_t[c] = b;
    }
}

template <typename T>
size_t fft_lds(int maxN, int maxL, bool third) {
    size_t off = sizeof(cpx<T>) * maxN * (third ? 3 : 2) + sizeof(cpx<T>) * maxL;
    off = (off + 7) & ~(size_t)7;
    return off + sizeof(double) * maxL + sizeof(double) * 4 * kWaves;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

unsigned grid_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Radix-order timing: every workgroup runs `reps` forward + inverse 2D FFTs of one L x L tile
// with the candidate plan, the same stage code and launch shape (kThreads per tile, LDS
// ping-pong) as the FFT kernels, rescaling by 1/N after each pair so nothing overflows.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fft_tune(const double* __restrict__ tw_tab,
                                                       RadixPlan rp, int L, int reps,
                                                       T* __restrict__ sink) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = L * L;
    cpx<T>* A = (cpx<T>*)smem;
    cpx<T>* S = A + N;
    cpx<T>* tw = S + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        A[i] = {T(1) / T(1 + (i + blockIdx.x) % 7), T(0)};
    for (int m = threadIdx.x; m < L; m += blockDim.x) tw[m] = {(T)tw_tab[2 * m], (T)tw_tab[2 * m + 1]};
    __syncthreads();
    const T scale = T(1) / T(N);
    for (int r = 0; r < reps; ++r) {
        fft2d<T, false>(A, S, L, rp, tw);
        fft2d<T, true>(A, S, L, rp, tw);
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            A[i].re *= scale;
            A[i].im *= scale;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = A[0].re;
}

template <typename T>
hipError_t time_fft_plan(const double* tw, const RadixPlan& rp, int L, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1, T* sink, unsigned blocks, float* ms_out) {
    constexpr int kReps = 8;
    const size_t lds = sizeof(cpx<T>) * (2 * (size_t)L * L + L);
    hipError_t e = allow_lds(k_fft_tune<T>, lds);
    float best = 1e30f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // the first launch only warms up
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_fft_tune<T>, dim3(blocks), dim3(kThreads), lds, s, tw, rp, L,
                               kReps, sink);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0) best = std::min(best, ms);
    }
    *ms_out = best;
    return e;
}

}  // namespace

hipError_t tune_radix_plan(fh_plan p, int L, const double* tw_dev, hipStream_t s,
                           RadixPlan* best, std::vector<TuneRecord>* log) {
    constexpr int kCap = 64;
    RadixPlan cand[kCap];
    const int n = radix_orders(L, cand, kCap);
    RadixPlan def;
    if (!default_radix_plan(L, &def)) return hipErrorInvalidValue;
    *best = def;
    if (n <= 1 || n > kCap) return hipSuccess;  // nothing to choose
    constexpr unsigned kBlocks = 1024;
    void* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&sink, kBlocks * sizeof(double));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best_ms = 1e30f, def_ms = 1e30f;
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        float ms = 0.0f;
        if (p->precision == FH_FP64)
            e = time_fft_plan<double>(tw_dev, cand[k], L, s, e0, e1, (double*)sink, kBlocks, &ms);
        else
            e = time_fft_plan<float>(tw_dev, cand[k], L, s, e0, e1, (float*)sink, kBlocks, &ms);
        if (e != hipSuccess) break;
        if (log) log->push_back({L, cand[k], ms});
        bool is_def = cand[k].n == def.n;
        for (int i = 0; i < def.n && is_def; ++i) is_def = cand[k].rad[i] == def.rad[i];
        if (is_def) def_ms = ms;
        if (ms < best_ms) {
            best_ms = ms;
            *best = cand[k];
        }
    }
    // the default stays unless a candidate is faster by more than 2%
    if (e != hipSuccess || !(best_ms < 0.98f * def_ms)) *best = def;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    return e;
}

size_t forward_lds_bytes(fh_plan p) {
    return p->precision == FH_FP64 ? fft_lds<double>(p->max_N, p->max_L, false)
                                   : fft_lds<float>(p->max_N, p->max_L, false);
}

size_t grad_lds_bytes(fh_plan p) {
    return p->precision == FH_FP64 ? fft_lds<double>(p->max_N, p->max_L, true)
                                   : fft_lds<float>(p->max_N, p->max_L, true);
}

hipError_t launch_set_sweep(fh_plan p, uint64_t sweep, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, p->d.sweep, sweep);
    return hipGetLastError();
}

hipError_t launch_bump_sweep(fh_plan p, hipStream_t s) {
    hipLaunchKernelGGL(k_bump_u64, dim3(1), dim3(64), 0, s, p->d.sweep);
    return hipGetLastError();
}

hipError_t launch_zero(void* ptr, int64_t bytes, hipStream_t s) {
    const int64_t words = bytes / 4;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(words)), dim3(kThreads), 0, s, (uint32_t*)ptr, words);
    return hipGetLastError();
}

hipError_t launch_potentials(fh_plan p, const void* aux, hipStream_t s) {
    const unsigned g = (unsigned)p->total_slices;
    if (p->precision == FH_FP64)
        hipLaunchKernelGGL(k_potentials<double>, dim3(g), dim3(kThreads), 0, s, p->d.chains,
                           p->n_chains, (const double*)aux, (double*)p->d.W, p->d.wshift,
                           p->aux_elems, p->total_slices, p->d.status);
    else
        hipLaunchKernelGGL(k_potentials<float>, dim3(g), dim3(kThreads), 0, s, p->d.chains,
                           p->n_chains, (const float*)aux, (float*)p->d.W, p->d.wshift,
                           p->aux_elems, p->total_slices, p->d.status);
    return hipGetLastError();
}

hipError_t launch_forward(fh_plan p, const void* aux, const int32_t* paths, hipStream_t s) {
    const size_t lds = forward_lds_bytes(p);
    hipError_t e;
    if (p->precision == FH_FP64) {
        if ((e = allow_lds(k_forward_fft<double>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_forward_fft<double>, dim3(p->n_fwd_tasks), dim3(kThreads), lds, s,
                           p->d.chains, p->d.fwd_tasks, p->d.tables, (const double*)aux,
                           (const double*)p->d.W,
                           p->d.wshift, p->aux_elems, p->total_slices, paths, p->d.perm, (double*)p->d.filt, p->d.blk_logz, p->d.sweep,
                           p->d.status, p->max_N, p->max_L, rescue_args(p));
    } else {
        if ((e = allow_lds(k_forward_fft<float>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_forward_fft<float>, dim3(p->n_fwd_tasks), dim3(kThreads), lds, s,
                           p->d.chains, p->d.fwd_tasks, p->d.tables, (const float*)aux,
                           (const float*)p->d.W,
                           p->d.wshift, p->aux_elems, p->total_slices, paths, p->d.perm, (float*)p->d.filt, p->d.blk_logz, p->d.sweep,
                           p->d.status, p->max_N, p->max_L, rescue_args(p));
    }
    return hipGetLastError();
}

hipError_t launch_logz_reduce(fh_plan p, double* logZ, hipStream_t s) {
    hipLaunchKernelGGL(k_logz_reduce, dim3((unsigned)((p->particles + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, p->d.chains, p->n_chains, p->d.blk_logz, logZ,
                       p->particles);
    return hipGetLastError();
}

namespace {
hipError_t launch_backward_kernels(fh_plan p, int32_t* paths, hipStream_t s) {
    if (p->n_draww_tasks > 0) {
        const unsigned blocks = (unsigned)((p->n_draww_tasks + kThreads / kWinLanes - 1) /
                                           (kThreads / kWinLanes));
        if (p->precision == FH_FP64)
            hipLaunchKernelGGL(k_backward_win<double>, dim3(blocks), dim3(kThreads), 0, s,
                               p->d.chains, p->d.draww_tasks, p->n_draww_tasks, p->d.tables,
                               (const double*)p->d.filt, paths, p->d.perm, p->d.sweep, p->d.status, p->d.bw_state,
                               p->bw_adapt ? 1 : 0, rescue_args(p), SlotRows{});
        else
            hipLaunchKernelGGL(k_backward_win<float>, dim3(blocks), dim3(kThreads), 0, s,
                               p->d.chains, p->d.draww_tasks, p->n_draww_tasks, p->d.tables,
                               (const float*)p->d.filt, paths, p->d.perm, p->d.sweep, p->d.status, p->d.bw_state,
                               p->bw_adapt ? 1 : 0, rescue_args(p), SlotRows{});
    }
    if (p->n_draw32_tasks > 0) {
        const unsigned blocks = (unsigned)((p->n_draw32_tasks + kWaves - 1) / kWaves);
        if (p->precision == FH_FP64)
            hipLaunchKernelGGL(k_backward_l32<double>, dim3(blocks), dim3(kThreads), 0, s,
                               p->d.chains, p->d.draw32_tasks, p->n_draw32_tasks, p->d.tables,
                               (const double*)p->d.filt, paths, p->d.perm, p->d.sweep, p->d.status, p->d.bw_state,
                               rescue_args(p));
        else
            hipLaunchKernelGGL(k_backward_l32<float>, dim3(blocks), dim3(kThreads), 0, s,
                               p->d.chains, p->d.draw32_tasks, p->n_draw32_tasks, p->d.tables,
                               (const float*)p->d.filt, paths, p->d.perm, p->d.sweep, p->d.status, p->d.bw_state,
                               rescue_args(p));
    }
    if (p->n_drawx_tasks == 0) return hipGetLastError();
    const unsigned blocks = (unsigned)((p->n_drawx_tasks + kWaves - 1) / kWaves);
    const DrawTask* tasks = p->d.drawx_tasks;
    const int n = p->n_drawx_tasks;
    if (p->max_N_x <= 1024) {
        if (p->precision == FH_FP64)
            hipLaunchKernelGGL(k_backward_fast<double>, dim3(blocks), dim3(kThreads), 0, s,
                               p->d.chains, tasks, n, p->d.tables, (const double*)p->d.filt, paths,
                               p->d.perm, p->d.sweep, p->d.status, p->d.bw_state,
                               rescue_args(p));
        else
            hipLaunchKernelGGL(k_backward_fast<float>, dim3(blocks), dim3(kThreads), 0, s,
                               p->d.chains, tasks, n, p->d.tables, (const float*)p->d.filt, paths,
                               p->d.perm, p->d.sweep, p->d.status, p->d.bw_state,
                               rescue_args(p));
        return hipGetLastError();
    }
    if (p->precision == FH_FP64)
        hipLaunchKernelGGL(k_backward<double>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           tasks, n, p->d.tables, (const double*)p->d.filt, paths, p->d.perm,
                           p->d.sweep, p->d.status, p->d.bw_state,
                               rescue_args(p));
    else
        hipLaunchKernelGGL(k_backward<float>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           tasks, n, p->d.tables, (const float*)p->d.filt, paths, p->d.perm,
                           p->d.sweep, p->d.status, p->d.bw_state,
                               rescue_args(p));
    return hipGetLastError();
}
}  // namespace

__global__ void k_scale_f32(float* __restrict__ dst, const float* __restrict__ src, int64_t n,
                            float factor) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] * factor;
}

hipError_t launch_scale_copy(float* dst, const float* src, int64_t n, float factor, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_f32, dim3(grid_for(n)), dim3(kThreads), 0, s, dst, src, n, factor);
    return hipGetLastError();
}

hipError_t launch_dedup(fh_plan p, const int32_t* paths, hipStream_t s) {
    if (p->n_dedup_tasks == 0 || p->share_off) return hipSuccess;
    hipLaunchKernelGGL(k_dedup, dim3((unsigned)p->n_dedup_tasks), dim3(kThreads), 0, s,
                       p->d.chains, p->d.dedup_tasks, paths, p->d.sweep, p->d.rep, rescue_args(p),
                       p->d.fwd32c_tasks, p->d.fwdxc_tasks, p->d.fwdpc_tasks, p->n_fwdp2_tasks,
                       p->d.prep);
    return hipGetLastError();
}

hipError_t launch_member_logz(fh_plan p, const int32_t* paths, hipStream_t s) {
    if (p->n_dedup_tasks == 0 || p->share_off) return hipSuccess;
    hipLaunchKernelGGL(k_member_logz, dim3(grid_for(p->blk_elems)), dim3(kThreads), 0, s,
                       p->d.chains, p->n_chains, paths, p->d.perm, p->d.sweep, p->d.blk_la,
                       p->d.endrow, p->d.blk_logz, p->blk_elems, p->d.status, rescue_args(p));
    return hipGetLastError();
}

hipError_t launch_rescue_reset(fh_plan p, hipStream_t s) {
    if (!p->d.rescue) return hipSuccess;
    hipLaunchKernelGGL(k_rescue_reset, dim3(grid_for(std::max<int64_t>(p->blk_elems, p->n_chains))),
                       dim3(kThreads), 0, s, rescue_args(p), p->blk_elems);
    return hipGetLastError();
}

hipError_t launch_rescue_expand(fh_plan p, hipStream_t s) {
    if (!p->d.rescue) return hipSuccess;
    hipLaunchKernelGGL(k_rescue_expand, dim3(p->n_chains), dim3(kThreads), 0, s, p->d.chains,
                       rescue_args(p));
    return hipGetLastError();
}

hipError_t launch_rescue_held(fh_plan p, hipStream_t s) {
    if (!p->d.rescue) return hipSuccess;
    hipLaunchKernelGGL(k_rescue_held, dim3(1), dim3(kThreads), 0, s, p->d.chains, rescue_args(p),
                       p->n_rescue_slots, (int)(p->n_dedup_tasks > 0 && !p->share_off),
                       p->d.arep);
    return hipGetLastError();
}

hipError_t launch_rescue(fh_plan p, const void* aux, int32_t* paths, bool draw, int phase,
                         hipStream_t s) {
    if (!p->d.rescue) return hipSuccess;
    hipLaunchKernelGGL(k_rescue_potentials, dim3((unsigned)p->total_slices), dim3(kThreads), 0, s,
                       p->d.chains, p->n_chains, (const float*)aux, p->d.wshift, p->d.rescue_w,
                       p->aux_elems, p->total_slices, rescue_args(p), phase);
    const unsigned blocks = (unsigned)(p->n_rescue_slots / kWaves);
    if (draw && phase == 1) {  // representatives into their slots, then every block's draws
        // L <= 32: a workgroup per representative; 48 x 48, 64 x 64: a wavefront each
        hipLaunchKernelGGL(k_rescue_share_fwd4, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->d.cmat64, (const float*)aux, p->d.wshift, p->total_slices, paths,
                           p->d.perm, p->d.blk_logz, p->d.blk_la, p->d.sweep, p->d.status,
                           rescue_args(p), p->d.arep, p->d.rep_slot, p->d.rescue_ws,
                           p->rescue_slot_elems, p->d.rescue_w, p->aux_elems);
        auto fwd = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                               p->d.cmat64, (const float*)aux, p->d.wshift, p->total_slices,
                               paths, p->d.perm, p->d.blk_logz, p->d.blk_la, p->d.sweep,
                               p->d.status, rescue_args(p), p->d.arep, p->d.rep_slot,
                               p->d.rescue_ws, p->rescue_slot_elems, p->n_rescue_slots,
                               p->d.rescue_w, p->aux_elems);
        };
        if (p->rescue_l64) fwd(k_rescue_share_fwd<4>);
        if (p->rescue_l48) fwd(k_rescue_share_fwd<3>);
        // the draws: windowed chains four blocks to a wavefront from the slots' FP64 rows, the
        // others one block to a wavefront (they take no slot: twice the slot count of them)
        const unsigned wblocks = (unsigned)((p->rescuable_blocks + kThreads / kWinLanes - 1) /
                                            (kThreads / kWinLanes));
        hipLaunchKernelGGL((k_backward_win<double, true>), dim3(wblocks), dim3(kThreads), 0, s,
                           p->d.chains, nullptr, 0, p->d.tables, nullptr, paths, p->d.perm,
                           p->d.sweep, p->d.status, p->d.bw_state, 0, rescue_args(p),
                           SlotRows{p->d.rep_slot, p->d.rescue_ws, p->rescue_slot_elems,
                                    p->d.blk_logz, p->d.blk_la});
        const int draw_waves = 2 * p->n_rescue_slots;
        hipLaunchKernelGGL(k_rescue_share_draw, dim3((unsigned)(draw_waves / kWaves)),
                           dim3(kThreads), 0, s, p->d.chains, p->d.tables, paths, p->d.perm,
                           p->d.blk_logz, p->d.blk_la, p->d.sweep, p->d.status, rescue_args(p),
                           p->d.rep_slot, p->d.rescue_ws, p->rescue_slot_elems, draw_waves);
    } else {
        // one launch per tiling: L <= 32, then the 64 x 64 and 48 x 48 chains, in stream order,
        // so the launches take the same slots in turn
        auto run = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                               p->d.tables, p->d.cmat64, (const float*)aux, p->d.wshift,
                               p->total_slices, paths, p->d.perm, (float*)p->d.filt,
                               p->d.blk_logz, p->d.sweep, p->d.status, rescue_args(p),
                               p->d.rescue_ws, p->rescue_slot_elems, p->n_rescue_slots,
                               p->d.rescue_w, p->aux_elems, phase);
        };
        if (draw) {
            run(k_rescue<true, 2>);
            if (p->rescue_l64) run(k_rescue<true, 4>);
            if (p->rescue_l48) run(k_rescue<true, 3>);
        } else {
            run(k_rescue<false, 2>);
            if (p->rescue_l64) run(k_rescue<false, 4>);
            if (p->rescue_l48) run(k_rescue<false, 3>);
        }
    }
    return hipGetLastError();
}

hipError_t launch_backward(fh_plan p, int32_t* paths, hipStream_t s) {
    // windowed draws where the hopping kernel allows them; 32 x 32 chains without the window (or
    // moved off it for this sweep by k_bw_adapt) on their own full-row kernel, the rest on the
    // generic ones
    hipError_t e = launch_backward_kernels(p, paths, s);
    if (e != hipSuccess || !p->bw_adapt || p->n_draww_tasks == 0) return e;
    hipLaunchKernelGGL(k_bw_adapt, dim3(1), dim3(kThreads), 0, s, p->d.chains, p->n_chains,
                       p->d.bw_state);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_local_t(fh_plan p, const T* aux, int32_t* paths, int n_passes, hipStream_t s) {
    const unsigned blocks = (unsigned)((p->particles + kThreads - 1) / kThreads);
    int max_tau = 2;
    for (const ChainInfo& c : p->chains) max_tau = std::max(max_tau, c.L_tau);
    const int pairs = std::max(1, (max_tau - 1) / 2);  // slice pairs of the interior phases
    constexpr int kMaxGridY = 65535;
    for (int ps = 0; ps < n_passes; ++ps) {
        for (int ph = 0; ph < 2; ++ph)
            for (int k0 = 0; k0 < pairs; k0 += kMaxGridY) {
                const dim3 grid(blocks, (unsigned)std::min(kMaxGridY, pairs - k0));
                if (ph == 0)
                    hipLaunchKernelGGL((k_local<T, 0>), grid, dim3(kThreads), 0, s, p->d.chains,
                                       p->n_chains, p->particles, p->d.tables, aux, paths,
                                       p->d.perm, p->d.perm_inv, p->d.sweep, ps, k0, p->d.status);
                else
                    hipLaunchKernelGGL((k_local<T, 1>), grid, dim3(kThreads), 0, s, p->d.chains,
                                       p->n_chains, p->particles, p->d.tables, aux, paths,
                                       p->d.perm, p->d.perm_inv, p->d.sweep, ps, k0, p->d.status);
            }
        hipLaunchKernelGGL((k_local<T, 2>), dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->n_chains, p->particles, p->d.tables, aux, paths, p->d.perm,
                           p->d.perm_inv, p->d.sweep, ps, 0, p->d.status);
        hipLaunchKernelGGL((k_local<T, 3>), dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->n_chains, p->particles, p->d.tables, aux, paths, p->d.perm,
                           p->d.perm_inv, p->d.sweep, ps, 0, p->d.status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_local(fh_plan p, const void* aux, int32_t* paths, int n_passes, hipStream_t s) {
    if (p->precision == FH_FP64) return launch_local_t(p, (const double*)aux, paths, n_passes, s);
    return launch_local_t(p, (const float*)aux, paths, n_passes, s);
}

hipError_t launch_perm_update(fh_plan p, const int32_t* paths, int n_passes, hipStream_t s) {
    const unsigned blocks = (unsigned)((p->particles + kThreads - 1) / kThreads);
    for (int ps = 0; ps < n_passes; ++ps) {
        hipLaunchKernelGGL(k_perm_update, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->n_chains, p->particles, p->d.tables, paths, p->d.perm,
                           p->d.perm_inv, p->d.sign, p->d.sweep, ps, p->d.status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t scratch_address(void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {  // once per device, with that device current
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_measure(fh_plan p, const int32_t* paths, double* Sk, double* Cr, double* D,
                          double* S2, hipStream_t s, double* work) {
    const size_t lds = sizeof(cpx<double>) * (2 * (size_t)p->max_N + p->max_L) +
                       sizeof(double) * 2 * kWaves;
    hipError_t e = allow_lds(k_measure, lds);
    if (e != hipSuccess) return e;
    double* sk = work;  // [aux_elems] S(k) rows, [aux_elems] C(r) rows, [2 slices] site sums
    double* cr = sk + p->aux_elems;
    double* sums = cr + p->aux_elems;
    hipLaunchKernelGGL(k_measure, dim3((unsigned)p->total_slices), dim3(kThreads), lds, s,
                       p->d.chains, p->n_chains, p->d.tables, paths, sk, cr, sums, p->d.status,
                       p->max_N, p->max_L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t n = p->total_sites + p->n_chains;
    hipLaunchKernelGGL(k_measure_reduce, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, p->d.chains, p->n_chains, p->total_sites, sk, cr,
                       sums, Sk, Cr, D, S2);
    return hipGetLastError();
}

hipError_t launch_mala_propose(fh_plan p, const void* aux, const void* dlogz, void* prop,
                               double eps, hipStream_t s) {
    const unsigned blocks = grid_for(p->aux_elems);
    if (p->precision == FH_FP64)
        hipLaunchKernelGGL(k_mala_propose<double>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->n_chains, p->aux_elems, (const double*)aux, (const double*)dlogz,
                           (double*)prop, eps, p->d.sweep);
    else
        hipLaunchKernelGGL(k_mala_propose<float>, dim3(blocks), dim3(kThreads), 0, s, p->d.chains,
                           p->n_chains, p->aux_elems, (const float*)aux, (const float*)dlogz,
                           (float*)prop, eps, p->d.sweep);
    return hipGetLastError();
}

hipError_t launch_mala_accept(fh_plan p, void* aux, const void* prop, const void* g0,
                              const void* g1, const double* logz0, const double* logz1,
                              double eps, int32_t* accepted, hipStream_t s) {
    if (p->precision == FH_FP64)
        hipLaunchKernelGGL(k_mala_accept<double>, dim3(p->n_chains), dim3(kThreads), 0, s,
                           p->d.chains, (double*)aux, (const double*)prop, (const double*)g0,
                           (const double*)g1, logz0, logz1, eps, p->d.sweep, accepted);
    else
        hipLaunchKernelGGL(k_mala_accept<float>, dim3(p->n_chains), dim3(kThreads), 0, s,
                           p->d.chains, (float*)aux, (const float*)prop, (const float*)g0,
                           (const float*)g1, logz0, logz1, eps, p->d.sweep, accepted);
    return hipGetLastError();
}

hipError_t launch_gibbs(fh_plan p, const int32_t* paths, void* aux, hipStream_t s) {
    const size_t lds = sizeof(int32_t) * 2 * p->max_N;
    if (p->precision == FH_FP64)
        hipLaunchKernelGGL(k_gibbs<double>, dim3((unsigned)p->total_slices), dim3(kThreads), lds,
                           s, p->d.chains, p->n_chains, paths, (double*)aux, p->d.sweep,
                           p->d.status, p->max_N);
    else
        hipLaunchKernelGGL(k_gibbs<float>, dim3((unsigned)p->total_slices), dim3(kThreads), lds,
                           s, p->d.chains, p->n_chains, paths, (float*)aux, p->d.sweep,
                           p->d.status, p->max_N);
    return hipGetLastError();
}

hipError_t launch_grad(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor,
                       void* grad_aux, hipStream_t s) {
    const size_t lds = grad_lds_bytes(p);
    hipError_t e;
    void* slabs = grad_aux ? p->d.gpart : nullptr;  // the field gradient only when asked for
    if (p->precision == FH_FP64) {
        if ((e = allow_lds(k_grad<double>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_grad<double>, dim3(p->n_groups), dim3(kThreads), lds, s,
                           p->d.chains, p->d.group_tasks, p->d.tables, (const double*)aux,
                           (const double*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, (double*)p->d.filt, p->d.blk_logz, p->d.dt, (double*)slabs,
                           anchor, p->d.perm, p->d.status, p->max_N, p->max_L);
    } else {
        if ((e = allow_lds(k_grad<float>, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_grad<float>, dim3(p->n_groups), dim3(kThreads), lds, s,
                           p->d.chains, p->d.group_tasks, p->d.tables, (const float*)aux,
                           (const float*)p->d.W, p->d.wshift, p->aux_elems, p->total_slices,
                           paths, (float*)p->d.filt, p->d.blk_logz, p->d.dt, (float*)slabs,
                           anchor, p->d.perm, p->d.status, p->max_N, p->max_L);
    }
    if ((e = hipGetLastError()) != hipSuccess || !grad_aux) return e;
    return launch_gpart_reduce(p, grad_aux, s);
}

__global__ void k_kinetic_scale(const ChainInfo* __restrict__ chains, int n_chains,
                                double* __restrict__ energy) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n_chains) {
        const ChainInfo& ci = chains[c];
        energy[c] *= -ci.hop_t / ((double)ci.L_tau * ci.dtau);
    }
}

hipError_t launch_kinetic_scale(fh_plan p, double* energy, hipStream_t s) {
    hipLaunchKernelGGL(k_kinetic_scale, dim3((unsigned)((p->n_chains + 63) / 64)), dim3(64), 0, s,
                       p->d.chains, p->n_chains, energy);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(fh_plan p, double* logZ, double* grad_t, hipStream_t s) {
    if (!logZ && !grad_t) return hipSuccess;
    hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)p->n_chains), dim3(64), 0, s,
                       p->d.chains, p->n_chains, p->d.blk_logz, p->d.dt, logZ, grad_t);
    return hipGetLastError();
}

}  // namespace fh
