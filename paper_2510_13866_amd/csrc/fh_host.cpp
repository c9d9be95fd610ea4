// Host side of the FFBS library: plan construction (validation, kernel tables, work lists,
// workspace), the C ABI entry points and hipGraph capture of a sweep.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "../../include/fh.h"
#include "../../include/fh_debug.h"
#include "fh_internal.h"
#include "fh_philox.h"

using namespace fh;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Modified Bessel function I_n(x), n >= 0, x >= 0, by its power series
// sum_k (x/2)^(2k+n) / (k! (k+n)!) — every term positive, so the sum keeps relative accuracy.
double bessel_i(int n, double x) {
    if (x == 0.0) return n == 0 ? 1.0 : 0.0;
    const double h = 0.5 * x;
    double term = exp(n * log(h) - lgamma((double)n + 1.0));
    double sum = term;
    for (int k = 0; k < 1000; ++k) {
        term *= h * h / ((k + 1.0) * (k + 1.0 + n));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

// g(d) = sum_{n = d (mod L)} I_n(2 t dtau): the inverse Fourier transform of
// exp(2 t dtau cos(2 pi m / L)) along one dimension (generating function of I_n).
void kernel_table(int L, double t, double dtau, double* g) {
    const double x = 2.0 * t * dtau;
    const int nmax = 3 * L + 40;
    for (int d = 0; d < L; ++d) g[d] = 0.0;
    for (int n = -nmax; n <= nmax; ++n) {
        int d = ((n % L) + L) % L;
        g[d] += bessel_i(n < 0 ? -n : n, x);
    }
}

void build_tables(const fh_chain_desc& d, double* tab) {
    const int L = d.L, N = L * L;
    std::vector<double> c(L);
    for (int m = 0; m < L; ++m) c[m] = cos(2.0 * kPi * m / L);
    for (int ky = 0; ky < L; ++ky)
        for (int kx = 0; kx < L; ++kx) {
            const double ck = c[kx] + c[ky];
            const double gh = exp(2.0 * d.t * d.dtau * ck);
            tab[kx + L * ky] = gh / N;                                // ghat / N
            tab[N + kx + L * ky] = 2.0 * d.dtau * ck * gh / N;        // d ghat / d t / N
        }
    kernel_table(L, d.t, d.dtau, tab + 2 * N);                        // g[L]
    double* tw = tab + 2 * N + L;                                     // exp(-2 pi i m / L)
    for (int m = 0; m < L; ++m) {
        tw[2 * m] = cos(2.0 * kPi * m / L);
        tw[2 * m + 1] = -sin(2.0 * kPi * m / L);
    }
}

uint16_t bf16_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

double bf16_val(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

// Split-bf16 operand of the circulant C[i][j] = g(i - j mod L) (zero outside L x L, 32 x 32
// tile) in the lane order the MFMA forward filter consumes: term t (x = h + m + l), K chunk q,
// lane, element e holds term_t(C[R][lane % 32]) with R = 16q + 8(e/4) + 4(lane/32) + e%4.
// B operands of the FP64 circulant for v_mfma_f64_16x16x4_f64: slot (4 K + r) * 2 + J, lane l
// holds C[16 K + 4 r + l / 16][16 J + l % 16], C[k][j] = g((k - j) mod L) inside L x L, else 0.
void build_cmat64(int L, const double* g, double* out) {
    if (const int NT = big_nt(L)) {  // block-circulant operands: entry 4 D + r
        for (int q = 0; q < 16; ++q)
            for (int lane = 0; lane < 64; ++lane) {
                const int D = q / 4, r = q % 4, k = lane / 16, j = lane % 16;
                out[q * 64 + lane] = D < NT ? g[((16 * D + 4 * r + k - j) % L + L) % L] : 0.0;
            }
        return;
    }
    for (int K = 0; K < 2; ++K)
        for (int r = 0; r < 4; ++r)
            for (int J = 0; J < 2; ++J)
                for (int lane = 0; lane < 64; ++lane) {
                    const int k = 16 * K + 4 * r + lane / 16, j = 16 * J + lane % 16;
                    out[((4 * K + r) * 2 + J) * 64 + lane] =
                        (L <= 32 && k < L && j < L) ? g[((k - j) % L + L) % L] : 0.0;
                }
}

// With bs < 32 the operand is block-diagonal: diagonal blocks of side bs, each holding the
// L x L circulant in its leading corner (the packed small-lattice forward); bs = 32 is the
// single padded circulant.
void build_cmat(int L, const double* g, uint16_t* out, int bs = 32) {
    if (L > bs) {
        memset(out, 0, sizeof(uint16_t) * kCmatPerChain);
        return;
    }
    for (int q = 0; q < 2; ++q)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                const int R = 16 * q + 8 * (e / 4) + 4 * (lane / 32) + e % 4;
                const int n = lane % 32;
                const int r = R % bs, k = n % bs;
                const double v = (R / bs == n / bs && r < L && k < L) ? g[((r - k) % L + L) % L] : 0.0;
                const uint16_t h = bf16_rne((float)v);
                const double r1 = v - bf16_val(h);
                const uint16_t m = bf16_rne((float)r1);
                const double r2 = r1 - bf16_val(m);
                const uint16_t l = bf16_rne((float)r2);
                const uint16_t terms[3] = {h, m, l};
                for (int t = 0; t < 3; ++t) out[((t * 2 + q) * 64 + lane) * 8 + e] = terms[t];
            }
}

// A 32 x 32 block C_KJ (rows 32 K .., columns 32 J ..) of the circulant g((i - j) mod L) of a
// lattice with 32 < L <= 64, zero-padded to 64 x 64, in the operand layout of build_cmat.
void build_cmat_block(int L, const double* g, int K, int J, uint16_t* out) {
    for (int q = 0; q < 2; ++q)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                const int R = 32 * K + 16 * q + 8 * (e / 4) + 4 * (lane / 32) + e % 4;
                const int n = 32 * J + lane % 32;
                const double v = (R < L && n < L) ? g[((R - n) % L + L) % L] : 0.0;
                const uint16_t h = bf16_rne((float)v);
                const double r1 = v - bf16_val(h);
                const uint16_t m = bf16_rne((float)r1);
                const double r2 = r1 - bf16_val(m);
                const uint16_t l = bf16_rne((float)r2);
                const uint16_t terms[3] = {h, m, l};
                for (int t = 0; t < 3; ++t) out[((t * 2 + q) * 64 + lane) * 8 + e] = terms[t];
            }
}

// The operand blocks of a chain with 32 < L <= 64 (kCmatPerChain values each, four per chain):
// L = 64 has two distinct blocks, C_00 = C_11 and C_01 = C_10 (-32 = 32 mod 64); a padded
// lattice has four, C_KJ at 2 K + J.
void build_cmat_blocks(int L, const double* g, uint16_t* out) {
    if (L <= 32 || L > 64) return;
    for (int b = 0; b < (L == 64 ? 2 : 4); ++b)
        build_cmat_block(L, g, b >> 1, b & 1, out + (size_t)kCmatPerChain * b);
}

bool is_fin(double v) { return std::isfinite(v); }

int validate(const fh_chain_desc& d, int precision) {
    RadixPlan rp;
    if (d.L < 2 || d.L_tau < 2 || d.n_up < 0 || d.n_dn < 0 || d.n_up + d.n_dn < 1)
        return FH_ERR_INVALID_ARG;
    if ((int64_t)d.n_up + d.n_dn > (int64_t)1 << 20) return FH_ERR_INVALID_ARG;
    if (d.L_tau > (1 << 20)) return FH_ERR_INVALID_ARG;
    if (d.hs_kind != FH_HS_GAUSS && d.hs_kind != FH_HS_HIRSCH) return FH_ERR_INVALID_ARG;
    if (!(d.block_len == 0 || (d.block_len >= 2 && d.block_len <= d.L_tau)))
        return FH_ERR_INVALID_ARG;
    if (!is_fin(d.t) || !is_fin(d.U) || !is_fin(d.dtau) || !(d.t > 0) || !(d.dtau > 0))
        return FH_ERR_INVALID_ARG;
    if (d.hs_kind == FH_HS_HIRSCH && d.U < 0) return FH_ERR_INVALID_ARG;
    if (!default_radix_plan(d.L, &rp)) return FH_ERR_UNSUPPORTED;
    return FH_OK;
}

// FP32 range parameters of a chain (see kRangeFloor): rows scaled by 2^row_exp, lowered from
// kRowExp when the kernel's mass sum G = exp(4 t dtau) exceeds 2^6, so that W~ 2^100 times a
// row of mass 2^row_exp stays below 2^126; the step floor is 2^-196 of a step's unweighted
// mass; a chain is queued whole when any of its blocks is queued.
void set_range(ChainInfo& ci, double t, double dtau, bool fp32) {
    ci.whole_min = 0;
    if (!fp32) {
        ci.row_exp = 0;
        ci.row_mass = 1.0;
        ci.step_floor = 0.0f;
        return;
    }
    const double lsum = 4.0 * t * dtau / log(2.0);  // log2 of sum_d G(d)
    ci.row_exp = kRowExp - std::max(0, (int)ceil(lsum) - 6);
    if (ci.row_exp < 0) ci.row_exp = 0;
    ci.row_mass = ldexp(1.0, ci.row_exp);
    ci.step_floor = (float)ldexp(exp(4.0 * t * dtau), ci.row_exp + kWScaleLog2 - 196);
}

template <typename T>
hipError_t dalloc(T** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    return hipMalloc((void**)p, bytes);
}

void free_device(fh::Device& d) {
    void* ptrs[] = {d.chains, d.tables, d.cmat, d.cmat64, d.fwdd_tasks, d.W, d.wshift, d.filt, d.blk_logz, d.dt, d.fwd_tasks,
                    d.draw_tasks, d.group_tasks, d.gpart, d.ckpt, d.rep, d.blk_la, d.endrow, d.dedup_tasks, d.fwd32_tasks, d.fwd32c_tasks, d.fwdxc_tasks, d.fwdpc_tasks, d.prep, d.fwdx_tasks, d.fwdp_tasks, d.cmatp, d.cmatb, d.fwd64_tasks, d.draw32_tasks, d.draww_tasks, d.drawx_tasks, d.meas, d.mala, d.perm, d.perm_inv, d.sign, d.bw_state,
                    d.rescue, d.rescue_list, d.rep_slot, d.arep, d.rescue_ws, d.rescue_w, d.status, d.sweep};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    d = fh::Device();
}

void drop_graph(fh_plan p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_aux = nullptr;
    p->graph_paths = nullptr;
}

int hip_status(hipError_t e) {
    if (e == hipSuccess) return FH_OK;
    if (e == hipErrorOutOfMemory) return FH_ERR_OOM;
    return FH_ERR_HIP;
}

#define FH_TRY(expr)                                 \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_status(_e); \
    } while (0)

}  // namespace

extern "C" {

const char* fh_strerror(int code) {
    switch (code) {
        case FH_OK: return "ok";
        case FH_ERR_INVALID_ARG: return "invalid argument";
        case FH_ERR_UNSUPPORTED: return "unsupported configuration";
        case FH_ERR_OOM: return "device out of memory";
        case FH_ERR_HIP: return "HIP runtime error";
        case FH_ERR_NONFINITE: return "non-finite weight or normaliser";
        case FH_ERR_ZERO_WEIGHT: return "zero total weight in backward sampling";
        case FH_ERR_STATE: return "call order violated";
        case FH_ERR_BAD_PATH: return "site index in paths out of range";
        default: return "unknown error";
    }
}

static void destroy_streams(fh_plan p) {
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    if (p->join_ev) (void)hipEventDestroy(p->join_ev);
}

int fh_init(fh_plan* out, const fh_chain_desc* descs, int32_t n_chains, int32_t precision,
            uint32_t flags) {
    if (!out) return FH_ERR_INVALID_ARG;
    *out = nullptr;
    if (!descs || n_chains < 1) return FH_ERR_INVALID_ARG;
    if (precision != FH_FP64 && precision != FH_FP32 && precision != FH_FP32_MFMA3)
        return FH_ERR_INVALID_ARG;
    if (flags & ~(uint32_t)(FH_FLAG_GRAPH | FH_FLAG_AUTOTUNE | FH_FLAG_FULL_ROW_DRAW |
                            FH_FLAG_FFT_CONV | FH_FLAG_GRAD_CHECKPOINT))
        return FH_ERR_INVALID_ARG;
    for (int c = 0; c < n_chains; ++c) {
        int v = validate(descs[c], precision);
        if (v != FH_OK) return v;
    }
    fh_plan p = new (std::nothrow) fh_plan_s();
    if (!p) return FH_ERR_OOM;
    p->n_chains = n_chains;
    p->precision = precision;
    p->flags = flags;
    p->real_size = precision == FH_FP64 ? 8 : 4;
    p->descs.assign(descs, descs + n_chains);

    int64_t aux = 0, path = 0, part = 0, tab = 0, filt = 0, blk = 0, slices = 0;
    for (int c = 0; c < n_chains; ++c) {
        const fh_chain_desc& d = descs[c];
        ChainInfo ci;
        memset(&ci, 0, sizeof(ci));
        ci.L = d.L;
        ci.N = d.L * d.L;
        ci.L_tau = d.L_tau;
        ci.n_up = d.n_up;
        ci.n_dn = d.n_dn;
        ci.np = d.n_up + d.n_dn;
        ci.hs_kind = d.hs_kind;
        ci.B = d.block_len == 0 ? d.L_tau : d.block_len;
        ci.nb = (d.L_tau + ci.B - 1) / ci.B;
        default_radix_plan(d.L, &ci.plan);
        ci.gauss_a = sqrt(fabs(d.U) * d.dtau);
        ci.dtau = d.dtau;
        ci.hop_t = d.t;
        ci.hirsch_lambda = d.hs_kind == FH_HS_HIRSCH ? acosh(exp(d.dtau * d.U / 2.0)) : 0.0;
        ci.coef_up = d.hs_kind == FH_HS_GAUSS ? ci.gauss_a : ci.hirsch_lambda;
        ci.coef_dn = d.hs_kind == FH_HS_GAUSS ? ci.gauss_a : -ci.hirsch_lambda;
        ci.seed = d.seed;
        ci.aux_off = aux;
        ci.path_off = path;
        ci.part_off = part;
        ci.tab_off = tab;
        ci.filt_off = filt;
        ci.blk_off = blk;
        ci.slice_off = slices;
        ci.site_off = p->total_sites;
        p->total_sites += ci.N;
        slices += d.L_tau;
        aux += (int64_t)d.L_tau * ci.N;
        path += (int64_t)d.L_tau * ci.np;
        part += ci.np;
        tab += tab_size(d.L);
        filt += (int64_t)ci.np * d.L_tau * ci.N;
        filt = (filt + 63) & ~(int64_t)63;  // every chain's filters start 256-byte aligned
        blk += (int64_t)ci.np * ci.nb;
        p->max_N = std::max(p->max_N, ci.N);
        p->max_L = std::max(p->max_L, ci.L);
        p->max_np = std::max(p->max_np, ci.np);
        p->chains.push_back(ci);
    }
    p->aux_elems = aux;
    p->path_elems = path;
    p->particles = part;
    p->blk_elems = blk;
    p->filt_elems = filt;
    p->total_slices = slices;
    p->tables.assign(tab, 0.0);
    p->cmat.assign((size_t)kCmatPerChain * n_chains, 0);
    p->cmatp.assign((size_t)kCmatPerChain * n_chains, 0);
    p->cmatb.assign((size_t)4 * kCmatPerChain * n_chains, 0);
    p->cmat64.assign((size_t)kCmat64PerChain * n_chains, 0.0);
    std::vector<char> windowed((size_t)n_chains, 0);
    for (int c = 0; c < n_chains; ++c) {
        ChainInfo& ci = p->chains[c];
        build_tables(descs[c], p->tables.data() + ci.tab_off);
        build_cmat(descs[c].L, p->tables.data() + tab_g(ci), p->cmat.data() + (size_t)kCmatPerChain * c);
        if (ci.L <= kPackMaxL)
            build_cmat(ci.L, p->tables.data() + tab_g(ci), p->cmatp.data() + (size_t)kCmatPerChain * c,
                       32 / pack_blocks(ci.L));
        build_cmat_blocks(ci.L, p->tables.data() + tab_g(ci),
                          p->cmatb.data() + (size_t)4 * kCmatPerChain * c);
        build_cmat64(descs[c].L, p->tables.data() + tab_g(ci),
                     p->cmat64.data() + (size_t)kCmat64PerChain * c);
        windowed[c] = win_select(p->tables.data() + tab_g(ci), ci.L, &ci.win_w, &ci.win_gout) &&
                      ci.L <= kWinMaxL && !(flags & FH_FLAG_FULL_ROW_DRAW);
        ci.win_on = windowed[c] ? 1 : 0;
        ci.win_gout2 = win_bound_for(p->tables.data() + tab_g(ci), ci.L, kWin2W);
        set_range(ci, descs[c].t, descs[c].dtau, precision != FH_FP64);
    }

    // Work lists, heaviest chains first so that the long tasks start early.
    std::vector<int> order(n_chains);
    for (int c = 0; c < n_chains; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const ChainInfo &x = p->chains[a], &y = p->chains[b];
        return (int64_t)x.B * x.N > (int64_t)y.B * y.N;
    });
    std::vector<PairTask> fwd;
    std::vector<DrawTask> draw;
    std::vector<GroupTask> groups;
    // the adjoint: FP64 circulant when every chain has L <= 32, else the FFT (one complex
    // signal = two worldlines per group); FP32 plans run the matrix-core adjoint
    p->grad_dmfma = precision == FH_FP64 && !(flags & FH_FLAG_FFT_CONV);
    for (const ChainInfo& ci : p->chains) p->grad_dmfma = p->grad_dmfma && ci.L <= 32;
    const bool mfma_grad = precision == FH_FP32_MFMA3 || p->grad_dmfma;
    // checkpoints are built into the matrix-core adjoints only (every chain with L <= 32)
    const bool ckpt = (flags & FH_FLAG_GRAD_CHECKPOINT) != 0;
    if (ckpt && !(mfma_grad && p->max_L <= 32)) {
        delete p;
        return FH_ERR_UNSUPPORTED;
    }
    const int gsize = mfma_grad ? kGroup : 2;
    int64_t gpart = 0, ck_rows = 0;
    for (int c = 0; c < n_chains; ++c) {  // checkpoint rows: ceil(L_tau / K) per worldline
        ChainInfo& ci = p->chains[c];
        ci.ck_k = (int32_t)ceil(sqrt((double)ci.L_tau));
        ci.ck_n = (ci.L_tau + ci.ck_k - 1) / ci.ck_k;
        ci.ck_row_off = ck_rows;
        ck_rows += (int64_t)ci.np * ci.ck_n * ci.N;
    }
    for (int c = 0; c < n_chains; ++c) {  // gradient groups in chain order (reduced per chain)
        ChainInfo& ci = p->chains[c];
        ci.g0 = (int32_t)groups.size();
        for (int spin = 0; spin < 2; ++spin) {
            int p0 = spin ? ci.n_up : 0, p1 = spin ? ci.np : ci.n_up;
            for (int q = p0; q < p1; q += gsize) {
                groups.push_back({c, q, std::min(gsize, p1 - q), spin, gpart, ck_rows});
                gpart += (int64_t)ci.L_tau * ci.N;
                ck_rows += (int64_t)kGroup * (ci.ck_k - 1) * ci.N;  // segment rows per wavefront
            }
        }
        ci.g1 = (int32_t)groups.size();
    }
    p->ckpt_elems = ckpt ? ck_rows : 0;
    for (int c : order) {
        const ChainInfo& ci = p->chains[c];
        for (int spin = 0; spin < 2; ++spin) {
            int p0 = spin ? ci.n_up : 0, p1 = spin ? ci.np : ci.n_up;
            for (int q = p0; q < p1; q += 2) {
                int qb = q + 1 < p1 ? q + 1 : -1;
                for (int b = 0; b < ci.nb; ++b) fwd.push_back({c, q, qb, b});
            }
        }
        for (int q = 0; q < ci.np; ++q)
            for (int b = 0; b < ci.nb; ++b) draw.push_back({c, q, b, 0});
    }
    // FP64 plans: chains with L <= 32 on the FP64 circulant, the others on the FFT
    auto dmfma = [&](int c) {
        return precision == FH_FP64 && !(flags & FH_FLAG_FFT_CONV) &&
               fp64_circulant(p->chains[c].L);
    };
    std::vector<PairTask> fwdf;
    // shared forward filters: the 32 x 32 chains of the matrix-core plan (one tile per worldline
    // pair) and its padded lattices (dedup = 1), and, in the FP64 re-filter of held chains only,
    // the 48 x 48 and 64 x 64 chains of FP32 plans (dedup = 2); k_dedup runs one workgroup per
    // (chain, spin, block)
    std::vector<DrawTask> dedup;
    for (int c = 0; c < n_chains; ++c) {
        ChainInfo& ci = p->chains[c];
        // the split-bf16 plan's chains with L <= 32: 32 x 32 tiles, padded lattices (16 < L < 32,
        // or small ones too large to pack), one tile per worldline, and packed small lattices
        const bool packs = ci.L <= kPackMaxL &&
                           (int64_t)ci.np * ci.L_tau * ci.N * 4 < ((int64_t)1 << 31);
        ci.pack = (precision == FH_FP32_MFMA3 && packs) ? pack_blocks(ci.L) : 0;
        ci.dedup = (precision == FH_FP32_MFMA3 && ci.L <= 32) ? 1
                   : (precision != FH_FP64 && big_nt(ci.L) != 0) ? 2 : 0;
        if (!ci.dedup) continue;
        if (ci.dedup == 1) {
            ci.end_off = p->end_elems;
            p->end_elems += (int64_t)ci.np * ci.nb * ci.N;
        }
        for (int spin = 0; spin < 2; ++spin)
            if ((spin ? ci.n_dn : ci.n_up) > 0)
                for (int b = 0; b < ci.nb; ++b) dedup.push_back({c, spin, b, 0});
    }
    p->n_dedup_tasks = (int32_t)dedup.size();
    std::vector<DrawTask> fwdd;
    for (const PairTask& t : fwd)
        if (!dmfma(t.chain)) fwdf.push_back(t);
    for (int nt : {2, 4, 3})  // L <= 32, then 64, then 48 (one launch each)
        for (const DrawTask& t : draw)
            if (dmfma(t.chain) && (nt == 2 ? p->chains[t.chain].L <= 32
                                           : big_nt(p->chains[t.chain].L) == nt)) {
                fwdd.push_back(t);
                (nt == 2 ? p->n_fwdd_tasks : nt == 4 ? p->n_fwdd4_tasks : p->n_fwdd3_tasks)++;
            }
    p->n_fwd_tasks = (int32_t)fwdf.size();
    p->n_draw_tasks = (int32_t)draw.size();
    std::vector<PairTask> fwd32;
    std::vector<DrawTask> fwdx, draw32, draww, drawx;
    std::vector<PackTask> fwdp2, fwdp4;
    std::vector<DrawTask> fwd64, fwd64p;
    // small lattices whose filter region (FP32) fits the packed kernel's 31-bit byte offsets
    auto packed = [&](int c) {
        const ChainInfo& ci = p->chains[c];
        return ci.L <= kPackMaxL && (int64_t)ci.np * ci.L_tau * ci.N * 4 < ((int64_t)1 << 31);
    };
    for (int c : order) {
        if (!packed(c)) continue;
        const ChainInfo& ci = p->chains[c];
        const int P = pack_blocks(ci.L), per = kPackTiles * P * P;
        for (int spin = 0; spin < 2; ++spin) {
            const int p0 = spin ? ci.n_up : 0, p1 = spin ? ci.np : ci.n_up;
            for (int q = p0; q < p1; q += per)
                for (int b = 0; b < ci.nb; ++b)
                    (P == 2 ? fwdp2 : fwdp4).push_back({c, q, std::min(per, p1 - q), b});
        }
    }
    for (const PairTask& t : fwd)
        if (p->chains[t.chain].L == 32) fwd32.push_back(t);
    // Backward: a windowed chain's tasks sit both in the windowed list and in a full-row list;
    // per sweep, bw_state decides which of the two kernels draws them (the other skips them).
    for (const DrawTask& t : draw) {
        if (p->chains[t.chain].L == 64) fwd64.push_back(t);
        else if (p->chains[t.chain].L > 32 && precision == FH_FP32_MFMA3) fwd64p.push_back(t);
        else if (p->chains[t.chain].L != 32 && !packed(t.chain) && p->chains[t.chain].L <= 32)
            fwdx.push_back(t);
        if (windowed[t.chain]) draww.push_back(t);
        else ++p->n_full_only_tasks;
        if (p->chains[t.chain].L == 32) {
            draw32.push_back(t);
        } else {
            drawx.push_back(t);
            p->max_N_x = std::max(p->max_N_x, p->chains[t.chain].N);
        }
    }
    p->n_fwd32_tasks = (int32_t)fwd32.size();
    p->n_fwdx_tasks = (int32_t)fwdx.size();
    p->n_fwdp2_tasks = (int32_t)fwdp2.size();
    p->n_fwd64_tasks = (int32_t)fwd64.size();
    p->n_fwd64p_tasks = (int32_t)fwd64p.size();
    fwd64.insert(fwd64.end(), fwd64p.begin(), fwd64p.end());  // the padded tasks follow
    p->n_fwdp4_tasks = (int32_t)fwdp4.size();
    std::vector<PackTask> fwdp(fwdp2);
    fwdp.insert(fwdp.end(), fwdp4.begin(), fwdp4.end());
    p->n_draw32_tasks = (int32_t)draw32.size();
    p->n_draww_tasks = (int32_t)draww.size();
    p->n_drawx_tasks = (int32_t)drawx.size();
    p->n_groups = (int32_t)groups.size();
    p->gpart_elems = gpart;

    // FP32 plans: the FP64 re-filter of blocks that leave FP32's range, one slot of FP64 rows
    // per wavefront, sized for the longest block of the chains it takes (L <= 32, 48, 64)
    if (precision != FH_FP64) {
        int64_t rescuable = 0;
        for (const ChainInfo& ci : p->chains)
            if (fp64_circulant(ci.L)) {
                p->rescue_l48 = p->rescue_l48 || ci.L == 48;
                p->rescue_l64 = p->rescue_l64 || ci.L == 64;
                // the block's rows and the end tile (phase A)
                p->rescue_slot_elems = std::max(p->rescue_slot_elems, (int64_t)ci.B * ci.N);
                rescuable += (int64_t)ci.np * ci.nb;
            }
        p->rescuable_blocks = rescuable;
        const int64_t waves = std::min<int64_t>(kRescueMaxSlots, std::max<int64_t>(rescuable, 1));
        p->n_rescue_slots = (int32_t)((waves + 3) / 4 * 4);
        p->rescue_slot_elems = std::max<int64_t>(p->rescue_slot_elems, 1);
    }

    hipError_t e = hipSuccess;
    fh::Device& dv = p->d;
    const size_t rs = p->real_size;
    if (e == hipSuccess) e = dalloc(&dv.chains, sizeof(ChainInfo) * n_chains);
    if (e == hipSuccess) e = dalloc(&dv.tables, sizeof(double) * p->tables.size());
    if (e == hipSuccess) e = dalloc(&dv.cmat, sizeof(uint16_t) * p->cmat.size());
    if (e == hipSuccess) e = dalloc(&dv.W, rs * 2 * (size_t)aux);
    if (e == hipSuccess) e = dalloc(&dv.wshift, sizeof(double) * 2 * (size_t)slices);
    if (e == hipSuccess && !ckpt) e = dalloc(&dv.filt, rs * (size_t)filt);
    if (e == hipSuccess && ckpt) e = dalloc(&dv.ckpt, rs * (size_t)p->ckpt_elems);
    if (e == hipSuccess) e = dalloc(&dv.blk_logz, sizeof(double) * (size_t)blk);
    if (e == hipSuccess && !dedup.empty()) {
        e = dalloc(&dv.rep, sizeof(int32_t) * (size_t)blk);
        if (e == hipSuccess) e = dalloc(&dv.blk_la, sizeof(double) * (size_t)blk);
        if (e == hipSuccess && p->end_elems > 0)
            e = dalloc(&dv.endrow, sizeof(float) * (size_t)p->end_elems);
        if (e == hipSuccess) e = dalloc(&dv.dedup_tasks, sizeof(DrawTask) * dedup.size());
        if (e == hipSuccess)
            e = hipMemcpy(dv.dedup_tasks, dedup.data(), sizeof(DrawTask) * dedup.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) {  // every worldline its own representative until k_dedup runs
            std::vector<int32_t> ident((size_t)blk);
            for (const ChainInfo& ci : p->chains)
                for (int64_t k = 0; k < (int64_t)ci.np * ci.nb; ++k)
                    ident[(size_t)(ci.blk_off + k)] = (int32_t)(k / ci.nb);
            e = hipMemcpy(dv.rep, ident.data(), sizeof(int32_t) * (size_t)blk,
                          hipMemcpyHostToDevice);
        }
    }
    if (e == hipSuccess) e = dalloc(&dv.dt, sizeof(double) * (size_t)part);
    if (e == hipSuccess) e = dalloc(&dv.fwd_tasks, sizeof(PairTask) * fwdf.size());
    if (e == hipSuccess) e = dalloc(&dv.fwdd_tasks, sizeof(DrawTask) * fwdd.size());
    if (e == hipSuccess) e = dalloc(&dv.cmat64, sizeof(double) * p->cmat64.size());
    if (e == hipSuccess) e = dalloc(&dv.draw_tasks, sizeof(DrawTask) * draw.size());
    if (e == hipSuccess) e = dalloc(&dv.group_tasks, sizeof(GroupTask) * groups.size());
    if (e == hipSuccess) e = dalloc(&dv.fwd32_tasks, sizeof(PairTask) * fwd32.size());
    if (e == hipSuccess && p->end_elems > 0 && !fwd32.empty())  // 32 x 32 chains share filters
        e = dalloc(&dv.fwd32c_tasks, sizeof(PairTask) * fwd32.size());
    if (e == hipSuccess && p->end_elems > 0 && !fwdx.empty())  // so do the padded lattices
        e = dalloc(&dv.fwdxc_tasks, sizeof(DrawTask) * fwdx.size());
    if (e == hipSuccess && p->end_elems > 0 && !fwdp.empty()) {  // and the packed ones
        int64_t n_prep = 0;
        for (const ChainInfo& ci : p->chains)
            if (ci.pack) n_prep += (int64_t)ci.np * ci.nb;
        e = dalloc(&dv.fwdpc_tasks, sizeof(PackTask) * fwdp.size());
        if (e == hipSuccess) e = dalloc(&dv.prep, sizeof(int32_t) * (size_t)n_prep);
    }
    if (e == hipSuccess) e = dalloc(&dv.fwdx_tasks, sizeof(DrawTask) * fwdx.size());
    if (e == hipSuccess) e = dalloc(&dv.fwdp_tasks, sizeof(PackTask) * fwdp.size());
    if (e == hipSuccess) e = dalloc(&dv.cmatp, sizeof(uint16_t) * p->cmatp.size());
    if (e == hipSuccess) e = dalloc(&dv.cmatb, sizeof(uint16_t) * p->cmatb.size());
    if (e == hipSuccess) e = dalloc(&dv.fwd64_tasks, sizeof(DrawTask) * fwd64.size());
    if (e == hipSuccess && !fwd64.empty()) e = hipMemcpy(dv.fwd64_tasks, fwd64.data(), sizeof(DrawTask) * fwd64.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = dalloc(&dv.draw32_tasks, sizeof(DrawTask) * draw32.size());
    if (e == hipSuccess) e = dalloc(&dv.draww_tasks, sizeof(DrawTask) * draww.size());
    if (e == hipSuccess) e = dalloc(&dv.drawx_tasks, sizeof(DrawTask) * drawx.size());
    if (e == hipSuccess) e = dalloc(&dv.gpart, p->real_size * (size_t)p->gpart_elems);
    if (e == hipSuccess) e = dalloc(&dv.perm, sizeof(int32_t) * (size_t)part);
    if (e == hipSuccess) e = dalloc(&dv.perm_inv, sizeof(int32_t) * (size_t)part);
    if (e == hipSuccess) e = dalloc(&dv.sign, sizeof(int32_t) * (size_t)n_chains);
    if (e == hipSuccess && p->n_rescue_slots > 0) {
        const size_t words = kRescueChain + kRescuePerChain * (size_t)n_chains + (size_t)blk;
        e = dalloc(&dv.rescue, sizeof(int32_t) * words);
        if (e == hipSuccess) e = hipMemset(dv.rescue, 0, sizeof(int32_t) * words);
        if (e == hipSuccess) e = dalloc(&dv.rescue_list, sizeof(DrawTask) * draw.size());
        if (e == hipSuccess) e = dalloc(&dv.rep_slot, sizeof(int32_t) * (size_t)blk);
        if (e == hipSuccess) e = dalloc(&dv.arep, sizeof(DrawTask) * (size_t)p->n_rescue_slots);
        if (e == hipSuccess && !ckpt)
            e = dalloc(&dv.rescue_ws, sizeof(double) * (size_t)p->n_rescue_slots * p->rescue_slot_elems);
        if (e == hipSuccess) e = dalloc(&dv.rescue_w, sizeof(double) * 2 * (size_t)aux);
    }
    if (e == hipSuccess) e = dalloc(&dv.status, sizeof(int32_t) * 2);
    if (e == hipSuccess) e = dalloc(&dv.bw_state, sizeof(int32_t) * (kBwCounts + (size_t)n_chains));
    if (e == hipSuccess) {
        std::vector<int32_t> zero(kBwCounts + (size_t)n_chains, 0);
        e = hipMemcpy(dv.bw_state, zero.data(), sizeof(int32_t) * zero.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = dalloc(&dv.sweep, sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemcpy(dv.tables, p->tables.data(), sizeof(double) * p->tables.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess && dv.rescue) {  // FP32 plans: phase A of the re-filter beside the sweep
        e = hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming);
    }
    // the static scratch of fh_measure_noalloc on this device: an address that cannot be taken
    // only disables that entry point
    if (e == hipSuccess && scratch_address(&p->scratch) != hipSuccess) {
        p->scratch = nullptr;
        (void)hipGetLastError();
    }
    if (e == hipSuccess && (flags & FH_FLAG_AUTOTUNE) && precision != FH_FP32_MFMA3) {
        // one timing sweep per distinct L, on the twiddles of its first chain (the FFT paths
        // only: the MFMA path has no radix plan)
        std::vector<int> done;
        for (int c = 0; c < n_chains && e == hipSuccess; ++c) {
            const int L = p->chains[c].L;
            if (std::find(done.begin(), done.end(), L) != done.end()) continue;
            done.push_back(L);
            RadixPlan best;
            e = tune_radix_plan(p, L, dv.tables + tab_tw(p->chains[c]), p->capture_stream, &best,
                                &p->tune_log);
            if (e == hipSuccess)
                for (ChainInfo& ci : p->chains)
                    if (ci.L == L) ci.plan = best;
        }
    }
    if (e == hipSuccess) e = hipMemcpy(dv.chains, p->chains.data(), sizeof(ChainInfo) * n_chains, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv.cmat, p->cmat.data(), sizeof(uint16_t) * p->cmat.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !fwdf.empty()) e = hipMemcpy(dv.fwd_tasks, fwdf.data(), sizeof(PairTask) * fwdf.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !fwdd.empty()) e = hipMemcpy(dv.fwdd_tasks, fwdd.data(), sizeof(DrawTask) * fwdd.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv.cmat64, p->cmat64.data(), sizeof(double) * p->cmat64.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv.draw_tasks, draw.data(), sizeof(DrawTask) * draw.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv.group_tasks, groups.data(), sizeof(GroupTask) * groups.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !fwd32.empty()) e = hipMemcpy(dv.fwd32_tasks, fwd32.data(), sizeof(PairTask) * fwd32.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !fwdx.empty()) e = hipMemcpy(dv.fwdx_tasks, fwdx.data(), sizeof(DrawTask) * fwdx.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !fwdp.empty()) e = hipMemcpy(dv.fwdp_tasks, fwdp.data(), sizeof(PackTask) * fwdp.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv.cmatp, p->cmatp.data(), sizeof(uint16_t) * p->cmatp.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dv.cmatb, p->cmatb.data(), sizeof(uint16_t) * p->cmatb.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !draw32.empty()) e = hipMemcpy(dv.draw32_tasks, draw32.data(), sizeof(DrawTask) * draw32.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !draww.empty()) e = hipMemcpy(dv.draww_tasks, draww.data(), sizeof(DrawTask) * draww.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !drawx.empty()) e = hipMemcpy(dv.drawx_tasks, drawx.data(), sizeof(DrawTask) * drawx.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) {  // every worldline closes on itself; sign +1
        std::vector<int32_t> id((size_t)part), one((size_t)n_chains, 1);
        for (const ChainInfo& ci : p->chains)
            for (int q = 0; q < ci.np; ++q) id[ci.part_off + q] = q;
        e = hipMemcpy(dv.perm, id.data(), sizeof(int32_t) * id.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(dv.perm_inv, id.data(), sizeof(int32_t) * id.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(dv.sign, one.data(), sizeof(int32_t) * one.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        int32_t st[2] = {0, -1};
        e = hipMemcpy(dv.status, st, sizeof(st), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        uint64_t z = 0;
        e = hipMemcpy(dv.sweep, &z, sizeof(z), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_device(dv);
        destroy_streams(p);
        delete p;
        (void)hipGetLastError();
        return hip_status(e);
    }
    *out = p;
    return FH_OK;
}

int fh_destroy(fh_plan p) {
    if (!p) return FH_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    drop_graph(p);
    for (hipEvent_t& ev : p->tev)
        if (ev) (void)hipEventDestroy(ev);
    free_device(p->d);
    destroy_streams(p);
    delete p;
    return FH_OK;
}

int fh_get_radix_plan(fh_plan p, int32_t chain, int32_t* radices, int32_t* n_stages) {
    if (!p || !radices || !n_stages || chain < 0 || chain >= p->n_chains) return FH_ERR_INVALID_ARG;
    const RadixPlan& rp = p->chains[chain].plan;
    *n_stages = rp.n;
    for (int i = 0; i < kMaxRadices; ++i) radices[i] = i < rp.n ? rp.rad[i] : 0;
    return FH_OK;
}

int fh_layout(fh_plan p, int32_t chain, fh_chain_layout* out) {
    if (!p || !out || chain < 0 || chain >= p->n_chains) return FH_ERR_INVALID_ARG;
    const ChainInfo& c = p->chains[chain];
    out->aux_offset = c.aux_off;
    out->aux_count = (int64_t)c.L_tau * c.N;
    out->path_offset = c.path_off;
    out->path_count = (int64_t)c.L_tau * c.np;
    out->particle_offset = c.part_off;
    out->L = c.L;
    out->N = c.N;
    out->L_tau = c.L_tau;
    out->n_particles = c.np;
    return FH_OK;
}

int fh_sizes(fh_plan p, int64_t* aux_elems, int64_t* path_elems, int64_t* particles) {
    if (!p) return FH_ERR_INVALID_ARG;
    if (aux_elems) *aux_elems = p->aux_elems;
    if (path_elems) *path_elems = p->path_elems;
    if (particles) *particles = p->particles;
    return FH_OK;
}

// Records timing event k of fh_debug_sweep_timing (no-op unless enabled).
static hipError_t mark(fh_plan p, int k, hipStream_t s) {
    return p->timing ? hipEventRecord(p->tev[k], s) : hipSuccess;
}

// The forward kernels of a pass, from the shared-filter map (unless the caller ran it) to the
// whole-chain queue.
static hipError_t enqueue_forward_kernels(fh_plan p, const void* aux, const int32_t* paths,
                                          hipStream_t s, bool dedup = true) {
    hipError_t e = mark(p, 0, s);
    if (e == hipSuccess && dedup) e = launch_dedup(p, paths, s);  // shared forward filters
    if (e != hipSuccess) return e;
    if (p->precision == FH_FP32_MFMA3) {
        e = launch_forward_mfma(p, aux, paths, s);
    } else {
        e = launch_forward_dmfma(p, aux, paths, s);  // FP64 plans: the FP64 circulant chains
        if (e == hipSuccess && p->n_fwd_tasks > 0) e = launch_forward(p, aux, paths, s);
    }
    if (e == hipSuccess) e = launch_member_logz(p, paths, s);
    if (e == hipSuccess) e = mark(p, 1, s);
    if (e == hipSuccess) e = launch_rescue_expand(p, s);  // FP32: chains re-filtered whole
    return e;
}

static hipError_t enqueue_forward(fh_plan p, const void* aux, const int32_t* paths, hipStream_t s) {
    hipError_t e = launch_potentials(p, aux, s);
    if (e == hipSuccess) e = launch_rescue_reset(p, s);  // FP32 plans: empty re-filter queue
    if (e == hipSuccess) e = enqueue_forward_kernels(p, aux, paths, s);
    return e;
}

// FH_FLAG_GRAD_CHECKPOINT plans allocate the filter workspace (and on FP32 plans the FP64
// re-filter's rows) at the first call that runs a forward filter, after the work queued on s:
// a plan used only for the adjoint never holds them.
static hipError_t ensure_filters(fh_plan p, hipStream_t s) {
    if (p->d.filt && (p->d.rescue_ws || !p->d.rescue)) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess && !p->d.filt)
        e = hipMalloc(&p->d.filt, p->real_size * (size_t)std::max<int64_t>(p->filt_elems, 1));
    if (e == hipSuccess && p->d.rescue && !p->d.rescue_ws)
        e = hipMalloc(&p->d.rescue_ws,
                      sizeof(double) * (size_t)p->n_rescue_slots * p->rescue_slot_elems);
    return e;
}

int fh_forward_filter(fh_plan p, const void* aux, const int32_t* paths, uint64_t sweep,
                      double* logZ, fh_stream stream) {
    if (!p || !aux || !paths) return FH_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    FH_TRY(ensure_filters(p, s));
    FH_TRY(launch_set_sweep(p, sweep, s));
    FH_TRY(enqueue_forward(p, aux, paths, s));
    FH_TRY(launch_rescue(p, aux, const_cast<int32_t*>(paths), false, 0, s));  // FP64 log Z, rows
    if (logZ) FH_TRY(launch_logz_reduce(p, logZ, s));
    p->have_filters = true;
    p->filters_are_ring = false;
    p->last_sweep = sweep;
    p->last_paths = paths;
    p->last_aux = aux;
    return FH_OK;
}

int fh_backward_sample(fh_plan p, int32_t* paths, uint64_t sweep, fh_stream stream) {
    if (!p || !paths) return FH_ERR_INVALID_ARG;
    if (!p->have_filters || p->filters_are_ring || sweep != p->last_sweep || paths != p->last_paths)
        return FH_ERR_STATE;
    hipStream_t s = (hipStream_t)stream;
    FH_TRY(launch_set_sweep(p, sweep, s));
    FH_TRY(launch_backward(p, paths, s));
    FH_TRY(launch_rescue(p, p->last_aux, paths, true, 0, s));  // blocks out of FP32's range
    return FH_OK;
}

int fh_gibbs_aux(fh_plan p, const int32_t* paths, void* aux, uint64_t sweep, fh_stream stream) {
    if (!p || !paths || !aux) return FH_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    FH_TRY(launch_set_sweep(p, sweep, s));
    FH_TRY(launch_gibbs(p, paths, aux, s));
    p->have_filters = false;
    return FH_OK;
}

int fh_local_update(fh_plan p, const void* aux, int32_t* paths, uint64_t sweep, int32_t n_passes,
                    fh_stream stream) {
    if (!p || !aux || !paths || n_passes < 0) return FH_ERR_INVALID_ARG;
    if (n_passes == 0) return FH_OK;
    hipStream_t s = (hipStream_t)stream;
    FH_TRY(launch_set_sweep(p, sweep, s));
    FH_TRY(launch_local(p, aux, paths, n_passes, s));
    p->have_filters = false;
    return FH_OK;
}

int fh_set_permutation(fh_plan p, const int32_t* perm) {
    if (!p || !perm) return FH_ERR_INVALID_ARG;
    std::vector<int32_t> h((size_t)p->particles), inv((size_t)p->particles), sg(p->n_chains);
    for (int c = 0; c < p->n_chains; ++c) {
        const ChainInfo& ci = p->chains[c];
        std::vector<char> seen(ci.np, 0);
        int cycles = 0;
        for (int q = 0; q < ci.np; ++q) {
            const int32_t v = perm[ci.part_off + q];
            const bool same_spin = (q < ci.n_up) == (v >= 0 && v < ci.n_up);
            if (v < 0 || v >= ci.np || !same_spin || seen[v]) return FH_ERR_INVALID_ARG;
            seen[v] = 1;
            h[ci.part_off + q] = v;
            inv[ci.part_off + v] = q;
        }
        std::vector<char> done(ci.np, 0);
        for (int q = 0; q < ci.np; ++q)
            if (!done[q]) {
                ++cycles;
                for (int r = q; !done[r]; r = h[ci.part_off + r]) done[r] = 1;
            }
        sg[c] = ((ci.np - cycles) % 2 == 0) ? 1 : -1;
    }
    FH_TRY(hipDeviceSynchronize());
    FH_TRY(hipMemcpy(p->d.perm, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice));
    FH_TRY(hipMemcpy(p->d.perm_inv, inv.data(), sizeof(int32_t) * inv.size(), hipMemcpyHostToDevice));
    FH_TRY(hipMemcpy(p->d.sign, sg.data(), sizeof(int32_t) * sg.size(), hipMemcpyHostToDevice));
    p->have_filters = false;
    return FH_OK;
}

int fh_get_permutation(fh_plan p, int32_t* perm, int32_t* sign) {
    if (!p) return FH_ERR_INVALID_ARG;
    FH_TRY(hipDeviceSynchronize());
    if (perm)
        FH_TRY(hipMemcpy(perm, p->d.perm, sizeof(int32_t) * (size_t)p->particles, hipMemcpyDeviceToHost));
    if (sign)
        FH_TRY(hipMemcpy(sign, p->d.sign, sizeof(int32_t) * (size_t)p->n_chains, hipMemcpyDeviceToHost));
    return FH_OK;
}

int fh_permutation_update(fh_plan p, const int32_t* paths, uint64_t sweep, int32_t n_passes,
                          fh_stream stream) {
    if (!p || !paths || n_passes < 0) return FH_ERR_INVALID_ARG;
    if (n_passes == 0) return FH_OK;
    hipStream_t s = (hipStream_t)stream;
    FH_TRY(launch_set_sweep(p, sweep, s));
    FH_TRY(launch_perm_update(p, paths, n_passes, s));
    p->have_filters = false;
    return FH_OK;
}

int fh_measure(fh_plan p, const int32_t* paths, double* Sk, double* Cr, double* D, double* S2,
               fh_stream stream) {
    if (!p || !paths) return FH_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (!p->d.meas) {  // first call: the per-slice rows
        const size_t n = 2 * (size_t)p->aux_elems + 2 * (size_t)p->total_slices;
        FH_TRY(hipStreamSynchronize(s));
        FH_TRY(hipMalloc((void**)&p->d.meas, sizeof(double) * n));
    }
    FH_TRY(launch_measure(p, paths, Sk, Cr, D, S2, s, p->d.meas));
    return FH_OK;
}

int fh_measure_noalloc(fh_plan p, const int32_t* paths, double* Sk, double* Cr, double* D,
                       double* S2, fh_stream stream) {
    if (!p || !paths) return FH_ERR_INVALID_ARG;
    if (2 * p->aux_elems + 2 * p->total_slices > kScratchDoubles) return FH_ERR_UNSUPPORTED;
    if (!p->scratch) return FH_ERR_HIP;  // its address could not be taken at fh_init
    FH_TRY(launch_measure(p, paths, Sk, Cr, D, S2, (hipStream_t)stream, (double*)p->scratch));
    return FH_OK;
}

// One sweep reading its index from the device word, as recorded into a graph.
// FP32 plans re-filter the chains held on FP64 (phase A) on the side stream, beside the FP32
// forward and backward passes of the other chains; the blocks those passes queue follow on the
// caller's stream once phase A has ended. The two touch disjoint chains: phase A writes the
// held chains' sites and block log Z, which the FP32 kernels skip (held at the pass start, or
// queued); the Gibbs draw reads every site after the join.
static hipError_t enqueue_sweep_body(fh_plan p, void* aux, int32_t* paths, hipStream_t s) {
    const bool split = p->side_stream != nullptr;
    hipError_t e = launch_potentials(p, aux, s);
    if (e == hipSuccess) e = launch_rescue_reset(p, s);
    // the shared-filter map first: phase A sizes by it and reads it beside the forward pass
    if (e == hipSuccess && split) e = launch_dedup(p, paths, s);
    if (split) {
        hipStream_t side = p->side_stream;
        if (e == hipSuccess) e = launch_rescue_held(p, s);
        if (e == hipSuccess) e = hipEventRecord(p->fork_ev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, p->fork_ev, 0);
        if (e == hipSuccess) e = mark(p, 5, side);
        if (e == hipSuccess) e = launch_rescue(p, aux, paths, true, 1, side);
        if (e == hipSuccess) e = mark(p, 6, side);
        if (e == hipSuccess) e = hipEventRecord(p->join_ev, side);
    }
    if (e == hipSuccess) e = enqueue_forward_kernels(p, aux, paths, s, !split);
    if (e == hipSuccess) e = mark(p, 2, s);
    if (e == hipSuccess) e = launch_backward(p, paths, s);
    if (e == hipSuccess) e = mark(p, 3, s);
    if (e == hipSuccess && split) e = hipStreamWaitEvent(s, p->join_ev, 0);
    if (e == hipSuccess) e = launch_rescue(p, aux, paths, true, split ? 2 : 0, s);
    if (e == hipSuccess) e = mark(p, 4, s);
    if (e == hipSuccess) e = launch_gibbs(p, paths, aux, s);
    return e;
}

static int capture_sweep(fh_plan p, void* aux, int32_t* paths) {
    drop_graph(p);
    hipStream_t cs = p->capture_stream;
    FH_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_sweep_body(p, aux, paths, cs);
    if (e == hipSuccess) e = launch_bump_sweep(p, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_status(e != hipSuccess ? e : e2);
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_status(e);
    }
    p->graph = g;
    p->graph_exec = ge;
    p->graph_aux = aux;
    p->graph_paths = paths;
    return FH_OK;
}

int fh_sweep(fh_plan p, void* aux, int32_t* paths, uint64_t first_sweep, int32_t n_sweeps,
             fh_stream stream) {
    if (!p || !aux || !paths || n_sweeps < 0) return FH_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n_sweeps == 0) return FH_OK;
    FH_TRY(ensure_filters(p, s));
    if ((p->flags & FH_FLAG_GRAPH) && !p->timing) {  // timed sweeps run eagerly (their events)
        if (!p->graph_exec || p->graph_aux != aux || p->graph_paths != paths) {
            // capture on the plan's stream after the caller's queued work is done
            FH_TRY(hipStreamSynchronize(s));
            int rc = capture_sweep(p, aux, paths);
            if (rc != FH_OK) return rc;
        }
        FH_TRY(launch_set_sweep(p, first_sweep, s));
        for (int32_t i = 0; i < n_sweeps; ++i) FH_TRY(hipGraphLaunch(p->graph_exec, s));
    } else {
        for (int32_t i = 0; i < n_sweeps; ++i) {
            FH_TRY(launch_set_sweep(p, first_sweep + (uint64_t)i, s));
            FH_TRY(enqueue_sweep_body(p, aux, paths, s));
        }
    }
    p->have_filters = false;
    return FH_OK;
}

static hipError_t enqueue_logz_grad(fh_plan p, const void* aux, const int32_t* paths,
                                    int32_t anchor_slice, double* logZ, void* grad_aux,
                                    double* grad_t, hipStream_t s) {
    hipError_t e = launch_potentials(p, aux, s);
    if (e != hipSuccess) return e;
    if (p->precision == FH_FP32_MFMA3) {
        e = launch_grad_mfma(p, aux, paths, anchor_slice, grad_aux, s);
    } else if (p->grad_dmfma) {
        e = launch_grad_dmfma(p, aux, paths, anchor_slice, grad_aux, s);
    } else {
        e = launch_grad(p, aux, paths, anchor_slice, grad_aux, s);
    }
    if (e == hipSuccess) e = launch_grad_reduce(p, logZ, grad_t, s);
    return e;
}

int fh_logZ_grad(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor_slice,
                 double* logZ, void* grad_aux, double* grad_t, fh_stream stream) {
    if (!p || !aux || !paths) return FH_ERR_INVALID_ARG;
    if (p->precision == FH_FP32_MFMA3 && p->max_L > 32) return FH_ERR_UNSUPPORTED;
    for (const ChainInfo& c : p->chains)
        if (anchor_slice < 0 || anchor_slice >= c.L_tau) return FH_ERR_INVALID_ARG;
    FH_TRY(enqueue_logz_grad(p, aux, paths, anchor_slice, logZ, grad_aux, grad_t,
                             (hipStream_t)stream));
    p->have_filters = p->d.ckpt == nullptr;  // with checkpoints the ring rows are not kept
    p->filters_are_ring = true;
    return FH_OK;
}

int fh_kinetic_energy(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor_slice,
                      double* energy, fh_stream stream) {
    if (!p || !aux || !paths || !energy) return FH_ERR_INVALID_ARG;
    if (p->precision == FH_FP32_MFMA3 && p->max_L > 32) return FH_ERR_UNSUPPORTED;
    for (const ChainInfo& c : p->chains)
        if (anchor_slice < 0 || anchor_slice >= c.L_tau) return FH_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    // d log Z_path / dt lands in energy (no field gradient, no log Z), then is scaled in place
    FH_TRY(enqueue_logz_grad(p, aux, paths, anchor_slice, nullptr, nullptr, energy, s));
    FH_TRY(launch_kinetic_scale(p, energy, s));
    p->have_filters = p->d.ckpt == nullptr;
    p->filters_are_ring = true;
    return FH_OK;
}

int fh_mala_field(fh_plan p, void* aux, const int32_t* paths, int32_t anchor_slice, double eps,
                  uint64_t sweep, int32_t* accepted, fh_stream stream) {
    if (!p || !aux || !paths || !(eps > 0.0) || !is_fin(eps)) return FH_ERR_INVALID_ARG;
    if (p->precision == FH_FP32_MFMA3 && p->max_L > 32) return FH_ERR_UNSUPPORTED;
    for (const ChainInfo& c : p->chains)
        if (anchor_slice < 0 || anchor_slice >= c.L_tau) return FH_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const size_t field = p->real_size * (size_t)p->aux_elems;
    if (!p->d.mala) {  // first call: proposal, two gradients, two log Z_path vectors
        FH_TRY(hipStreamSynchronize(s));
        FH_TRY(hipMalloc(&p->d.mala, 3 * field + 2 * sizeof(double) * (size_t)p->n_chains));
    }
    char* base = (char*)p->d.mala;
    void* prop = base;
    void* g0 = base + field;
    void* g1 = base + 2 * field;
    double* lz0 = (double*)(base + 3 * field);
    double* lz1 = lz0 + p->n_chains;
    FH_TRY(launch_set_sweep(p, sweep, s));
    FH_TRY(enqueue_logz_grad(p, aux, paths, anchor_slice, lz0, g0, nullptr, s));
    FH_TRY(launch_mala_propose(p, aux, g0, prop, eps, s));
    FH_TRY(enqueue_logz_grad(p, prop, paths, anchor_slice, lz1, g1, nullptr, s));
    FH_TRY(launch_mala_accept(p, aux, prop, g0, g1, lz0, lz1, eps, accepted, s));
    p->have_filters = false;
    return FH_OK;
}

int fh_set_hopping(fh_plan p, const double* t) {
    if (!p || !t) return FH_ERR_INVALID_ARG;
    for (int c = 0; c < p->n_chains; ++c)
        if (!is_fin(t[c]) || !(t[c] > 0)) return FH_ERR_INVALID_ARG;
    FH_TRY(hipDeviceSynchronize());
    for (int c = 0; c < p->n_chains; ++c) {
        ChainInfo& ci = p->chains[c];
        p->descs[c].t = t[c];
        ci.hop_t = t[c];
        build_tables(p->descs[c], p->tables.data() + ci.tab_off);
        build_cmat(p->descs[c].L, p->tables.data() + tab_g(ci),
                   p->cmat.data() + (size_t)kCmatPerChain * c);
        if (ci.L <= kPackMaxL)
            build_cmat(ci.L, p->tables.data() + tab_g(ci), p->cmatp.data() + (size_t)kCmatPerChain * c,
                       32 / pack_blocks(ci.L));
        build_cmat_blocks(ci.L, p->tables.data() + tab_g(ci),
                          p->cmatb.data() + (size_t)4 * kCmatPerChain * c);
        build_cmat64(p->descs[c].L, p->tables.data() + tab_g(ci),
                     p->cmat64.data() + (size_t)kCmat64PerChain * c);
        // the window keeps its width; its outside bound follows the new kernel
        ci.win_gout = win_bound_for(p->tables.data() + tab_g(ci), ci.L, ci.win_w) *
                      p->win_bound_scale;
        ci.win_gout2 = win_bound_for(p->tables.data() + tab_g(ci), ci.L, kWin2W) *
                       p->win_bound_scale;
        set_range(ci, t[c], p->descs[c].dtau, p->precision != FH_FP64);
    }
    FH_TRY(hipMemcpy(p->d.chains, p->chains.data(), sizeof(ChainInfo) * p->n_chains,
                     hipMemcpyHostToDevice));
    FH_TRY(hipMemcpy(p->d.tables, p->tables.data(), sizeof(double) * p->tables.size(),
                     hipMemcpyHostToDevice));
    FH_TRY(hipMemcpy(p->d.cmat, p->cmat.data(), sizeof(uint16_t) * p->cmat.size(),
                     hipMemcpyHostToDevice));
    FH_TRY(hipMemcpy(p->d.cmatp, p->cmatp.data(), sizeof(uint16_t) * p->cmatp.size(),
                     hipMemcpyHostToDevice));
    FH_TRY(hipMemcpy(p->d.cmatb, p->cmatb.data(), sizeof(uint16_t) * p->cmatb.size(),
                     hipMemcpyHostToDevice));
    FH_TRY(hipMemcpy(p->d.cmat64, p->cmat64.data(), sizeof(double) * p->cmat64.size(),
                     hipMemcpyHostToDevice));
    p->have_filters = false;
    return FH_OK;
}

int fh_get_status(fh_plan p, int32_t* code, int32_t* first_chain) {
    if (!p) return FH_ERR_INVALID_ARG;
    FH_TRY(hipDeviceSynchronize());
    int32_t st[2];
    FH_TRY(hipMemcpy(st, p->d.status, sizeof(st), hipMemcpyDeviceToHost));
    int32_t clear[2] = {0, -1};
    FH_TRY(hipMemcpy(p->d.status, clear, sizeof(clear), hipMemcpyHostToDevice));
    if (code) *code = st[0];
    if (first_chain) *first_chain = st[0] == 0 ? -1 : st[1];
    return FH_OK;
}

int fh_get_filters(fh_plan p, int32_t chain, int32_t particle, void* dst, int64_t capacity,
                   int64_t* n_rows, fh_stream stream) {
    if (!p || chain < 0 || chain >= p->n_chains) return FH_ERR_INVALID_ARG;
    const ChainInfo& c = p->chains[chain];
    if (particle < 0 || particle >= c.np) return FH_ERR_INVALID_ARG;
    if (!p->have_filters || !p->d.filt) return FH_ERR_STATE;
    const int64_t rows = p->filters_are_ring ? c.L_tau : c.L_tau - c.nb;
    if (n_rows) *n_rows = rows;
    if (!dst) return FH_OK;
    if (capacity < rows * c.N) return FH_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    // sweep rows of a chain with shared forward filters: block b's rows are its
    // representative's
    std::vector<int32_t> owner((size_t)c.nb, particle);
    if (!p->filters_are_ring && c.dedup && p->d.rep) {
        FH_TRY(hipStreamSynchronize(s));
        FH_TRY(hipMemcpy(owner.data(), p->d.rep + c.blk_off + (int64_t)particle * c.nb,
                         sizeof(int32_t) * c.nb, hipMemcpyDeviceToHost));
    }
    // ring rows: one block of L_tau rows; sweep rows: B - 1 (the last block: its length - 1)
    const int nseg = p->filters_are_ring ? 1 : c.nb;
    int64_t done = 0;
    for (int b = 0; b < nseg; ++b) {
        const int64_t cnt = p->filters_are_ring ? rows
                          : (b < c.nb - 1 ? c.B : c.L_tau - (int64_t)(c.nb - 1) * c.B) - 1;
        const int64_t from = c.filt_off + ((int64_t)owner[(size_t)b] * c.L_tau +
                                           (int64_t)b * (c.B - 1)) * c.N;
        const char* src = (const char*)p->d.filt + p->real_size * (size_t)from;
        char* to = (char*)dst + p->real_size * (size_t)(done * c.N);
        if (cnt > 0) {
            if (!p->filters_are_ring && c.row_exp != 0)  // FP32 sweep rows hold f~ 2^row_exp
                FH_TRY(launch_scale_copy((float*)to, (const float*)src, cnt * c.N,
                                         (float)ldexp(1.0, -c.row_exp), s));
            else
                FH_TRY(hipMemcpyAsync(to, src, p->real_size * (size_t)(cnt * c.N),
                                      hipMemcpyDeviceToDevice, s));
        }
        done += cnt;
    }
    FH_TRY(hipStreamSynchronize(s));
    return FH_OK;
}

// ---- host-only diagnostics ----------------------------------------------------------------

namespace {
// The device kernels' 2D Stockham FFT, run on the host over every butterfly.
void fft2d_host(double* data, int L, const RadixPlan& rp, bool inverse) {
    const int N = L * L;
    std::vector<cpx<double>> a(N), b(N), tw(L);
    for (int i = 0; i < N; ++i) a[i] = {data[2 * i], data[2 * i + 1]};
    for (int m = 0; m < L; ++m) tw[m] = {cos(2.0 * kPi * m / L), -sin(2.0 * kPi * m / L)};
    cpx<double>* src = a.data();
    cpx<double>* dst = b.data();
    for (int dim = 0; dim < 2; ++dim) {
        const int ls = dim == 0 ? L : 1, es = dim == 0 ? 1 : L;
        int Ns = 1;
        for (int st = 0; st < rp.n; ++st) {
            const int pr = rp.rad[st];
            for (int bf = 0; bf < L * (L / pr); ++bf) {
                if (inverse)
                    stockham_butterfly_rt<double, true>(pr, bf, L, Ns, ls, es, src, dst, tw.data());
                else
                    stockham_butterfly_rt<double, false>(pr, bf, L, Ns, ls, es, src, dst, tw.data());
            }
            Ns *= pr;
            std::swap(src, dst);
        }
    }
    for (int i = 0; i < N; ++i) {
        data[2 * i] = src[i].re;
        data[2 * i + 1] = src[i].im;
    }
}
}  // namespace

int fh_debug_fft2d_host(double* data, int32_t L, int32_t inverse) {
    RadixPlan rp;
    if (!data || !default_radix_plan(L, &rp)) return FH_ERR_UNSUPPORTED;
    fft2d_host(data, L, rp, inverse != 0);
    return FH_OK;
}

int fh_debug_fft2d_host_plan(double* data, int32_t L, const int32_t* radices, int32_t n_stages,
                             int32_t inverse) {
    if (!data || !radices || n_stages < 1 || n_stages > kMaxRadices) return FH_ERR_INVALID_ARG;
    RadixPlan rp;
    rp.n = n_stages;
    for (int i = 0; i < kMaxRadices; ++i) rp.rad[i] = i < n_stages ? radices[i] : 0;
    if (!valid_radix_plan(L, rp)) return FH_ERR_INVALID_ARG;
    fft2d_host(data, L, rp, inverse != 0);
    return FH_OK;
}

int fh_debug_radix_orders(int32_t L, int32_t* out, int32_t cap) {
    if (cap < 0 || (cap > 0 && !out)) return FH_ERR_INVALID_ARG;
    std::vector<RadixPlan> v(cap > 0 ? cap : 1);
    const int n = radix_orders(L, v.data(), cap);
    for (int k = 0; k < std::min(n, (int)cap); ++k) {
        out[7 * k] = v[k].n;
        for (int i = 0; i < kMaxRadices; ++i) out[7 * k + 1 + i] = i < v[k].n ? v[k].rad[i] : 0;
    }
    return n;
}

int fh_debug_kernel_table(int32_t L, double t, double dtau, double* out) {
    if (!out || L < 2 || L > kMaxL || !(t > 0) || !(dtau > 0)) return FH_ERR_INVALID_ARG;
    kernel_table(L, t, dtau, out);
    return FH_OK;
}

int fh_debug_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                    uint64_t* out) {
    if (!out) return FH_ERR_INVALID_ARG;
    u64x4 r = philox4x64_10(c0, c1, c2, c3, k0, k1);
    out[0] = r.x0;
    out[1] = r.x1;
    out[2] = r.x2;
    out[3] = r.x3;
    return FH_OK;
}

int fh_debug_window_select(const double* g, int32_t L, int32_t* w, double* g_out) {
    if (!g || !w || !g_out || L < 2 || L > kMaxL) return FH_ERR_INVALID_ARG;
    int ww = 0;
    double go = 0.0;
    const bool ok = win_select(g, L, &ww, &go);
    *w = ww;
    *g_out = go;
    return ok ? 1 : 0;
}

int fh_debug_window_draw(int32_t L, int32_t w, const double* g, double g_out, const double* f,
                         int32_t s_site, double u, int32_t* site, int32_t* certified) {
    if (!g || !f || !site || !certified || L < 2 || L > kMaxL || w < 1 || w > kWinMaxW ||
        s_site < 0 || s_site >= L * L || !(u >= 0.0 && u < 1.0) || !(g_out >= 0.0))
        return FH_ERR_INVALID_ARG;
    const int N = L * L;
    const int cx = s_site % L, cy = s_site / L;
    auto wt = [&](int x, int y) {
        int dx = cx - x, dy = cy - y;
        dx += dx < 0 ? L : 0;
        dy += dy < 0 ? L : 0;
        const double fi = f[x + L * y];
        return (fi > 0.0 ? fi : 0.0) * (g[dy] * g[dx]);
    };
    // a window of half-width ww: its cumulative weights in rank (= site) order, then the
    // certificate against the outside bound go
    auto try_window = [&](int ww, double go) {
        const int WW = win_width(ww, L), nwin = WW * WW;
        std::vector<double> P(nwin);
        std::vector<int> xs(nwin), ys(nwin);
        double acc = 0.0;
        for (int q = 0; q < nwin; ++q) {
            xs[q] = win_coord(q % WW, cx, ww, L, WW);
            ys[q] = win_coord(q / WW, cy, ww, L, WW);
            acc += wt(xs[q], ys[q]);
            P[q] = acc;
        }
        const double T_in = acc, tau = u * T_in;
        if (!(T_in > 0.0) || !std::isfinite(T_in)) return -1;
        int q = 0;
        while (q < nwin && !(P[q] > tau)) ++q;
        if (q < nwin && win_certified(q ? P[q - 1] : 0.0, P[q], tau,
                                      go * kWinMassBound + kWinSlack * T_in))
            return xs[q] + L * ys[q];
        return -1;
    };
    int r = try_window(w, g_out);
    if (r >= 0) {
        *certified = 1;
        *site = r;
        return FH_OK;
    }
    r = try_window(kWin2W, win_bound_for(g, L, kWin2W));
    if (r >= 0) {
        *certified = 2;
        *site = r;
        return FH_OK;
    }
    *certified = 0;
    // the full row in site order: first cumulative weight above u * total, else the last
    // positive weight
    double total = 0.0;
    for (int i = 0; i < N; ++i) total += wt(i % L, i / L);
    if (!std::isfinite(total)) return FH_ERR_NONFINITE;
    if (!(total > 0.0)) return FH_ERR_ZERO_WEIGHT;
    const double T = u * total;
    double run = 0.0;
    int last = -1;
    for (int i = 0; i < N; ++i) {
        const double wi = wt(i % L, i / L);
        run += wi;
        if (run > T) {
            *site = i;
            return FH_OK;
        }
        if (wi > 0.0) last = i;
    }
    *site = last;
    return FH_OK;
}

int fh_debug_inflate_window_bound(fh_plan p, double factor) {
    if (!p || !(factor >= 1.0)) return FH_ERR_INVALID_ARG;
    FH_TRY(hipDeviceSynchronize());
    p->win_bound_scale = factor;
    for (ChainInfo& ci : p->chains) {
        ci.win_gout = win_bound_for(p->tables.data() + tab_g(ci), ci.L, ci.win_w) * factor;
        ci.win_gout2 = win_bound_for(p->tables.data() + tab_g(ci), ci.L, kWin2W) * factor;
    }
    FH_TRY(hipMemcpy(p->d.chains, p->chains.data(), sizeof(ChainInfo) * p->n_chains,
                     hipMemcpyHostToDevice));
    return FH_OK;
}

int fh_debug_backward_kernels(fh_plan p, int32_t* n_windowed, int32_t* n_full_row) {
    if (!p || !n_windowed || !n_full_row) return FH_ERR_INVALID_ARG;
    *n_windowed = p->n_draww_tasks;
    *n_full_row = p->n_full_only_tasks;
    return FH_OK;
}

int fh_debug_backward_adapt(fh_plan p, int32_t enable, int32_t* full_row_passes_left) {
    if (!p || (enable != 0 && enable != 1)) return FH_ERR_INVALID_ARG;
    FH_TRY(hipDeviceSynchronize());
    std::vector<int32_t> st(kBwCounts + (size_t)p->n_chains);
    FH_TRY(hipMemcpy(st.data(), p->d.bw_state, sizeof(int32_t) * st.size(), hipMemcpyDeviceToHost));
    if (full_row_passes_left) *full_row_passes_left = st[0];
    if ((enable != 0) != p->bw_adapt) {
        p->bw_adapt = enable != 0;
        drop_graph(p);  // the captured sweep launches the adaptation kernel or not
        std::fill(st.begin(), st.end(), 0);  // back on the window
        FH_TRY(hipMemcpy(p->d.bw_state, st.data(), sizeof(int32_t) * st.size(), hipMemcpyHostToDevice));
    }
    return FH_OK;
}

int fh_debug_rescue(fh_plan p, int32_t* last_count, int32_t* whole_chains, int64_t* total,
                    int32_t* list, int32_t cap) {
    if (!p || cap < 0 || (cap > 0 && !list)) return FH_ERR_INVALID_ARG;
    if (last_count) *last_count = 0;
    if (whole_chains) *whole_chains = 0;
    if (total) *total = 0;
    if (!p->d.rescue) return FH_OK;
    FH_TRY(hipDeviceSynchronize());
    int32_t w[3];
    FH_TRY(hipMemcpy(w, p->d.rescue, sizeof(w), hipMemcpyDeviceToHost));
    const int32_t zero = 0;
    FH_TRY(hipMemcpy(p->d.rescue + 1, &zero, sizeof(zero), hipMemcpyHostToDevice));
    if (last_count) *last_count = w[0];
    if (whole_chains) *whole_chains = w[2];
    if (total) *total = w[1];
    const int n = std::min(cap, w[0]);
    if (n > 0) {
        std::vector<DrawTask> t((size_t)n);
        FH_TRY(hipMemcpy(t.data(), p->d.rescue_list, sizeof(DrawTask) * n, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) {
            list[3 * i] = t[i].chain;
            list[3 * i + 1] = t[i].p;
            list[3 * i + 2] = t[i].block;
        }
    }
    return FH_OK;
}

int fh_debug_fill_filter_row(fh_plan p, int32_t chain, int32_t particle, int32_t row,
                             double value) {
    if (!p || chain < 0 || chain >= p->n_chains) return FH_ERR_INVALID_ARG;
    const ChainInfo& c = p->chains[chain];
    if (particle < 0 || particle >= c.np) return FH_ERR_INVALID_ARG;
    if (!p->have_filters || !p->d.filt) return FH_ERR_STATE;
    const int64_t rows = p->filters_are_ring ? c.L_tau : c.L_tau - c.nb;
    if (row < 0 || row >= rows) return FH_ERR_INVALID_ARG;
    FH_TRY(hipDeviceSynchronize());
    const size_t off = (size_t)(c.filt_off + ((int64_t)particle * c.L_tau + row) * c.N);
    if (p->real_size == 8) {
        std::vector<double> v((size_t)c.N, value);
        FH_TRY(hipMemcpy((double*)p->d.filt + off, v.data(), sizeof(double) * c.N,
                         hipMemcpyHostToDevice));
    } else {
        std::vector<float> v((size_t)c.N, (float)value);
        FH_TRY(hipMemcpy((float*)p->d.filt + off, v.data(), sizeof(float) * c.N,
                         hipMemcpyHostToDevice));
    }
    return FH_OK;
}

int fh_debug_share_filters(fh_plan p, int32_t enable) {
    if (!p || (enable != 0 && enable != 1)) return FH_ERR_INVALID_ARG;
    if (!p->d.rep) return FH_OK;
    FH_TRY(hipDeviceSynchronize());
    drop_graph(p);  // the captured sweep holds the sharing kernels or not
    p->share_off = enable == 0;
    if (p->share_off) {  // every worldline its own representative
        std::vector<int32_t> ident((size_t)p->blk_elems);
        for (const ChainInfo& ci : p->chains)
            for (int64_t k = 0; k < (int64_t)ci.np * ci.nb; ++k)
                ident[(size_t)(ci.blk_off + k)] = (int32_t)(k / ci.nb);
        FH_TRY(hipMemcpy(p->d.rep, ident.data(), sizeof(int32_t) * ident.size(),
                         hipMemcpyHostToDevice));
    }
    p->have_filters = false;
    return FH_OK;
}

int fh_debug_representatives(fh_plan p, int32_t* rep, int64_t cap, int64_t* n) {
    if (!p || cap < 0 || (cap > 0 && !rep)) return FH_ERR_INVALID_ARG;
    if (n) *n = p->d.rep ? p->blk_elems : 0;
    if (!p->d.rep || cap == 0) return FH_OK;
    FH_TRY(hipDeviceSynchronize());
    FH_TRY(hipMemcpy(rep, p->d.rep, sizeof(int32_t) * (size_t)std::min(cap, p->blk_elems),
                     hipMemcpyDeviceToHost));
    return FH_OK;
}

int fh_debug_rescue_holds(fh_plan p, int32_t* holds) {
    if (!p || !holds) return FH_ERR_INVALID_ARG;
    std::fill(holds, holds + p->n_chains, 0);
    if (!p->d.rescue) return FH_OK;
    FH_TRY(hipDeviceSynchronize());
    FH_TRY(hipMemcpy(holds, p->d.rescue + kRescueChain + p->n_chains,
                     sizeof(int32_t) * p->n_chains, hipMemcpyDeviceToHost));
    return FH_OK;
}

int fh_debug_rescue_causes(fh_plan p, int32_t* counts) {
    if (!p || !counts) return FH_ERR_INVALID_ARG;
    std::fill(counts, counts + 4, 0);
    if (!p->d.rescue) return FH_OK;
    FH_TRY(hipDeviceSynchronize());
    FH_TRY(hipMemcpy(counts, p->d.rescue + kRescueCause, sizeof(int32_t) * 4,
                     hipMemcpyDeviceToHost));
    return FH_OK;
}

int fh_debug_sweep_timing(fh_plan p, int32_t enable) {
    if (!p || (enable != 0 && enable != 1)) return FH_ERR_INVALID_ARG;
    FH_TRY(hipDeviceSynchronize());
    if (enable && !p->tev[0])
        for (hipEvent_t& ev : p->tev) FH_TRY(hipEventCreate(&ev));
    p->timing = enable != 0;
    return FH_OK;
}

int fh_debug_sweep_times(fh_plan p, float* ms) {
    if (!p || !ms || !p->timing) return FH_ERR_INVALID_ARG;
    FH_TRY(hipEventSynchronize(p->tev[4]));
    for (int k = 0; k < 3; ++k) {
        const int a = k == 0 ? 0 : k + 1;
        FH_TRY(hipEventElapsedTime(&ms[k], p->tev[a], p->tev[a + 1]));
    }
    ms[3] = 0.0f;
    if (p->side_stream) FH_TRY(hipEventElapsedTime(&ms[3], p->tev[5], p->tev[6]));
    return FH_OK;
}

int fh_debug_forward_kernels(fh_plan p, int32_t* counts) {
    if (!p || !counts) return FH_ERR_INVALID_ARG;
    counts[0] = p->n_fwd32_tasks;
    counts[1] = p->n_fwdx_tasks;
    counts[2] = p->n_fwdp2_tasks;
    counts[3] = p->n_fwdp4_tasks;
    counts[4] = p->n_fwd64_tasks;
    counts[5] = p->n_fwd64p_tasks;
    return FH_OK;
}

}  // extern "C"
