// Internal declarations shared by the host API (fh_host.cpp) and the kernels (fh_kernels.hip,
// fh_mfma.hip). Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <utility>
#include <vector>

#include "../../include/fh.h"
#include "fh_fft.h"
#include "fh_window.h"

namespace fh {

// Per-chain parameters and offsets as the kernels see them (plain data, copied to the device).
struct ChainInfo {
    int32_t L, N, L_tau, n_up, n_dn, np, hs_kind, B, nb;
    RadixPlan plan;           // FFT radix plan of one dimension (both dimensions are L)
    double coef_up, coef_dn;  // log W_spin = coef_spin * aux
    double gauss_a, hirsch_lambda, dtau, hop_t;
    uint64_t seed;
    int64_t aux_off;   // packed aux / W offset (elements): aux[aux_off + l*N + r]
    int64_t path_off;  // packed paths offset: paths[path_off + l*np + p]
    int64_t part_off;  // per-particle arrays (logZ, dt)
    int64_t tab_off;   // double tables: ghat[N]/N, dghat[N]/N, g[L], tw[2L]
    int64_t filt_off;  // filter workspace: filt[filt_off + (p*L_tau + row)*N + r]
    int64_t blk_off;   // per-(particle, block) log Z: blk[blk_off + p*nb + block]
    int64_t slice_off; // index of this chain's slice 0 among all chains' slices
    int64_t site_off;  // per-site outputs (S(k), C(r)) packed by chain: [site_off + r]
    int32_t g0, g1;    // gradient worldline groups of this chain: [g0, g1)
    int32_t win_w;     // windowed backward draws: half-width w of the window around s
    int32_t win_on;    // 1: the chain's draws may use the windowed kernel (see bw_state)
    double win_gout;   // bound on G(s - r) over the sites r outside that window
    double win_gout2;  // the same for the second window (half-width kWin2W)
    // FP32 plans: the forward rows of the sweep hold f~ 2^row_exp (row mass 2^row_exp instead
    // of 1) and a block is queued for the FP64 re-filter when a step's W-weighted mass falls
    // below step_floor (see kRangeFloor). FP64 plans: row_exp = 0, row_mass = 1.
    int32_t row_exp;
    float step_floor;
    double row_mass;
    int32_t whole_min;  // queued blocks of one pass above which the whole chain is queued
    // FH_FLAG_GRAD_CHECKPOINT: the adjoint keeps ring rows j = 0, K, 2K, .. (K = ck_k =
    // ceil(sqrt(L_tau)), ck_n = ceil(L_tau / K) of them per worldline) at
    // ckpt[ck_row_off + (p ck_n + j / K) N] and recomputes each segment from its checkpoint
    int64_t ck_row_off;
    int32_t ck_k, ck_n;
    // Shared forward filters: the rows of a block depend only on the spin's W and the block's
    // start site, so worldlines of one (spin, block) with the same start site share the rows of
    // the lowest-numbered of them, their representative. dedup = 1: every chain with L <= 32 of
    // the split-bf16 plan (32 x 32, padded and packed tiles), in the FP32 passes and the FP64
    // re-filter's phase A; end_off locates their per-(particle, block) end tiles [N].
    // dedup = 2: 48 x 48 and 64 x 64 chains of FP32 plans,
    // in phase A only (their FP32 passes keep one recursion per worldline, and their map is the
    // identity while the chain is not held).
    int32_t dedup;
    int32_t pack;  // the packed forward's P (4: L <= 8, 2: L <= 16) on the split-bf16 plan, else 0
    int64_t end_off;
};

// Offsets of the tables of one chain inside the double table buffer, relative to tab_off.
FH_HD inline int64_t tab_ghat(const ChainInfo& c) { return c.tab_off; }
FH_HD inline int64_t tab_dghat(const ChainInfo& c) { return c.tab_off + c.N; }
FH_HD inline int64_t tab_g(const ChainInfo& c) { return c.tab_off + 2 * c.N; }
FH_HD inline int64_t tab_tw(const ChainInfo& c) { return c.tab_off + 2 * c.N + c.L; }
inline int64_t tab_size(int L) { return 2 * (int64_t)L * L + L + 2 * L; }
constexpr int kBwCounts = 4;  // offset of the per-chain counts in Device::bw_state
constexpr int kCmatPerChain = 3 * 2 * 64 * 8;
constexpr int kCmat64PerChain = 16 * 64;
// Lattices above 32 that the FP64 circulant takes (fh_dmfma.h): L = 16 NT with NT = 3 or 4; 0
// for every other L.
FH_HD inline int big_nt(int L) { return L == 48 ? 3 : L == 64 ? 4 : 0; }
// Chains whose blocks the FP64 re-filter can redo (L <= 32 or a big_nt lattice).
FH_HD inline bool fp64_circulant(int L) { return L <= 32 || big_nt(L) != 0; }

// Block of a sweep: start slice and length (the schedule of fh.h).
FH_HD inline void block_of(const ChainInfo& c, uint64_t sweep, int b, int* start, int* len) {
    const int o = (int)(((sweep % (uint64_t)c.L_tau) * (uint64_t)(c.B / 2)) % (uint64_t)c.L_tau);
    *start = (o + b * c.B) % c.L_tau;
    *len = (b < c.nb - 1) ? c.B : c.L_tau - (c.nb - 1) * c.B;
}

// Work items. Forward / gradient pairs share (chain, spin): p_b < 0 means a single particle.
struct PairTask {
    int32_t chain, p_a, p_b, block;
};
struct DrawTask {
    int32_t chain, p, block, pad;
};
// Worldlines p0 .. p0 + n - 1 of one (chain, spin), one block: the packed small-lattice forward
// (kPackTiles tiles of P x P worldlines, n <= kPackTiles P^2).
struct PackTask {
    int32_t chain, p0, n, block;
};
// Lattices up to this size run the packed forward: P = 4 blocks per tile side for L <= 8,
// P = 2 for L <= 16.
constexpr int kPackMaxL = 16;
FH_HD inline int pack_blocks(int L) { return L <= 8 ? 4 : 2; }
// Tiles per wavefront of the packed forward. One tile (P^2 worldlines) per wavefront measured
// faster than two on batches of mixed block lengths (finer work items balance better) and
// within 5% on uniform ones.
constexpr int kPackTiles = 1;
// Up to kGroup worldlines of one (chain, spin) processed by one workgroup in the matrix-core
// adjoints (two, one complex FFT signal, in the FFT adjoint); part_off locates the group's
// partial field-gradient slab [L_tau][N], which k_gpart_reduce adds per chain in a fixed order.
constexpr int kGroup = 4;
struct GroupTask {
    int32_t chain, p0, count, spin;
    int64_t part_off;
    int64_t seg_off;  // FH_FLAG_GRAD_CHECKPOINT: the group's segment rows [kWaves][K - 1][N]
};

// FP32 range. FP32 holds a value to full relative precision only down to ~2^-126, and the
// three-term bf16 split of the matrix-core forward only down to ~2^-110, while the weights of
// strongly clustered fields span far more than that. The FP32 plans therefore place both
// operands of the weight multiply high in FP32's range: W tables hold W~ 2^kWScaleLog2
// (W~ = W / max_r W of the slice, so the table's largest entry is 2^100 and W~ down to 2^-226
// is representable), and forward rows hold f~ 2^row_exp (row mass 2^20). A block is queued for
// the FP64 re-filter and redraw (k_rescue) when what its draws need approaches the floor: a
// forward step whose W-weighted mass is below 2^-196 of its unweighted mass (step_floor: the
// weights FP32 flushed to zero can then matter), an end weight below kRangeFloor = 2^-90
// (2^-110 of the row mass; it also needs the far hops of the circulant, whose bf16 terms stop
// there), or a backward draw that picks a site whose FP32 filter value is below kRangeFloor or
// finds no positive weight (the draw's FP64 weights carry G exactly, so only the filter value
// is in question). When a chain has a block queued in a forward pass (more than
// whole_min), every block of the chain is re-filtered in FP64 in that pass and in the next
// kRescueHold forward passes, which skip the chain's FP32 work: on the way to a clustered state
// many blocks meet a floor and some FP32 blocks drift without meeting one (a hop whose product
// underflows in one slice can move log Z by 16 nats), while the blocks of a settled chain meet a
// floor all together or not at all. When its hold has run out, a chain runs FP32 again to see
// whether it still needs FP64; each such retry that fails doubles the next hold, up to
// kRescueHoldMax passes, and a pass that needs no FP64 resets it to kRescueHold (k_rescue_reset).
constexpr int kWScaleLog2 = 100;
constexpr int kRowExp = 20;
constexpr float kRangeFloor = 0x1p-90f;
constexpr double kRangeFloorD = 0x1p-90;
constexpr int kRescueHold = 4;
constexpr int kRescueHoldMax = 64;
// Size of the static scratch array of fh_measure_noalloc: 2^22 doubles (32 MiB) per GPU.
constexpr int64_t kScratchDoubles = (int64_t)1 << 22;
// Rescue state words: [0] blocks queued in this pass, [1] blocks redrawn since the last read by
// fh_debug_rescue, [2] chains re-filtered whole in this pass, [3] length of the queue's phase A
// (a sweep's held chains, queued before its FP32 forward pass and re-filtered beside the FP32
// passes), [4] slots taken by phase A, [5] entries of the dense list of representative pairs
// (k_dedup), [6] entries of phase A's dense list of representatives (k_rescue_held), [7] entries
// of the dense list of the padded lattices' representatives (k_dedup), [8] and [9] entries of
// the dense lists of packed tiles of representatives (P = 2 and P = 4, k_dedup), [10]
// representatives listed for those tiles, [11 + k] the blocks queued for floor k since the
// plan was made (kCause*: never cleared, read by fh_debug_rescue_causes), [15] unused, then per
// chain: blocks queued by the kernels in this pass
// (kRescueChain + c), forward passes left on FP64 (kRescueChain + n_chains + c), 1 if the chain
// is in phase A (kRescueChain + 2 n_chains + c), the forward recursions its blocks need in this
// pass (kRescueChain + 3 n_chains + c: the representatives of the shared filters), the hold at
// the start of the previous pass (kRescueChain + 4 n_chains + c) and the length of the next
// hold (kRescueChain + 5 n_chains + c), then one flag per (chain, particle, block) at
// kRescueChain + kRescuePerChain n_chains + blk_off + p nb + b (the `flags` pointer passed to
// the kernels).
constexpr int kRescueChain = 16;
// Why a kernel queued a block (rescue words 11 + cause): a forward step's W-weighted mass below
// step_floor (or not finite), an end weight below kRangeFloor, a backward draw at a site whose
// filter value is below kRangeFloor (or with no positive weight), an FFT forward (either floor).
constexpr int kRescueCause = 11;
constexpr int kCauseStep = 0, kCauseEnd = 1, kCauseDraw = 2, kCauseFft = 3;
constexpr int kRescuePerChain = 6;
// XCDs of the MI355X; a launch deals its workgroups to them in turn.
constexpr int kXcds = 8;
// Slots of the FP64 re-filter (two wavefronts per SIMD of 256 CUs), (B - 1) N doubles of rows
// plus the end tile [N]. Phase 0 and 2 give each wavefront its own slot; phase A gives each
// representative one (k_rescue_held admits held chains while their representatives fit).
constexpr int kRescueMaxSlots = 2048;
constexpr int kDedupMaxN = 4096;  // sites of the largest chain with shared filters (64 x 64)
// Phase A's draws need no slot of their own: k_rescue_share_draw keeps this many wavefronts per
// SIMD (its register budget) and is launched with twice the slot count of them.
constexpr int kShareDrawWaves = 4;
// Shared forward filters: a chain whose representatives' rows (this pass) take at most this many
// bytes writes them with cached stores, the rest with nontemporal ones.
constexpr int64_t kCachedRowBytes = 16ll << 20;

// Per-pass state of the FP32 plans as the kernels see it: the rescue words above, the per-block
// flags, the queue, and the representative map of the shared forward filters (rep, per
// (chain, particle, block) at blk_off + p nb + b: the worldline whose stored rows the block's
// draws read; null where no chain shares, and on FP64 plans).
// Phase A's FP64 rows as the windowed backward kernel reads them when it draws the held chains'
// blocks (k_backward_win with SLOT): the slot of each representative's block, the slots, and the
// log Z pieces of the worldlines that share a representative's rows.
struct SlotRows {
    const int32_t* rep_slot;
    const double* ws;
    int64_t slot_elems;
    double* blk_logz;
    const double* blk_la;
};
struct Rescue {
    int32_t* words;   // null for FP64 plans
    int32_t* flags;   // words + kRescueChain + kRescuePerChain n_chains
    DrawTask* list;
    int32_t n_chains;
    const int32_t* rep;
};
// The worldline whose stored rows block `block` of worldline p reads.
__device__ inline int row_owner(const Rescue& r, const ChainInfo& c, int p, int block) {
    return r.rep ? r.rep[c.blk_off + (int64_t)p * c.nb + block] : p;
}
// Queues block (chain, p, block) for the FP64 re-filter once; called by one lane.
__device__ inline bool rescue_enqueue(const Rescue& r, const ChainInfo& c, int chain, int p,
                                      int block) {
    if (atomicExch(&r.flags[c.blk_off + (int64_t)p * c.nb + block], 1) != 0) return false;
    const int i = atomicAdd(&r.words[0], 1);
    r.list[i] = DrawTask{chain, p, block, 0};
    return true;
}
// A kernel found block (chain, p, block) out of FP32's range: queue it, count it for its chain
// and hold the chain on the FP64 re-filter for the next kRescueHold forward passes, or longer
// after failed retries (k_rescue_reset; a backward pass queues after the chain's blocks were
// expanded for this one).
__device__ inline void rescue_push(const Rescue& r, const ChainInfo& c, int chain, int p,
                                   int block, int cause) {
    atomicAdd(&r.words[kRescueCause + cause], 1);
    if (rescue_enqueue(r, c, chain, p, block)) {
        atomicAdd(&r.words[kRescueChain + chain], 1);
        atomicMax(&r.words[kRescueChain + r.n_chains + chain], kRescueHold);
    }
}
__device__ inline bool rescue_queued(const Rescue& r, const ChainInfo& c, int p, int block) {
    return r.words && r.flags[c.blk_off + (int64_t)p * c.nb + block] != 0;
}
// The chain is held on the FP64 re-filter for this forward pass (k_rescue_expand queues it
// whole whatever the FP32 pass finds): the FP32 forward kernels of chains with L <= 32 skip its
// tasks.
__device__ inline bool rescue_held(const Rescue& r, int chain) {
    return r.words && r.words[kRescueChain + r.n_chains + chain] > 0;
}

// One autotuner timing: the radix order `plan` of lattice size L took `ms` per timing launch.
struct TuneRecord {
    int32_t L;
    RadixPlan plan;
    float ms;
};

struct Device {
    ChainInfo* chains = nullptr;
    double* tables = nullptr;
    uint16_t* cmat = nullptr;  // per chain: split-bf16 circulant operand [3][2][64][8]
    uint16_t* cmatp = nullptr; // per chain with L <= kPackMaxL: the block-diagonal operand, same layout
    uint16_t* cmatb = nullptr; // per chain with 32 < L <= 64: four blocks C_KJ (L = 64: C_00, C_01), same layout
    double* cmat64 = nullptr;  // per chain: FP64 circulant B operands [16][64]
    DrawTask* fwdd_tasks = nullptr;  // FP64 circulant forward: worldline blocks (L <= 32, 48, 64)
    void* W = nullptr;        // [2][sum L_tau*N] in plan precision (up, then down)
    double* wshift = nullptr; // [2][total slices]: log W = log W~ + wshift per (spin, slice)
    void* filt = nullptr;     // filter workspace, plan precision
    double* blk_logz = nullptr;
    // shared forward filters (chains with dedup): representative map [blk_elems], the
    // representatives' log Z before the end weight [blk_elems], end tiles [end_elems] f32, and
    // the (chain, spin, block) tasks of k_dedup
    int32_t* rep = nullptr;
    double* blk_la = nullptr;
    float* endrow = nullptr;
    DrawTask* dedup_tasks = nullptr;
    double* dt = nullptr;     // per particle d log Z / d t
    PairTask* fwd_tasks = nullptr;
    DrawTask* draw_tasks = nullptr;
    GroupTask* group_tasks = nullptr;
    PairTask* fwd32_tasks = nullptr;    // MFMA forward: worldline pairs of L = 32 chains
    PairTask* fwd32c_tasks = nullptr;   // the dense representative pairs k_dedup lists (as many)
    DrawTask* fwdxc_tasks = nullptr;    // the same for the padded lattices' single worldlines
    DrawTask* fwdx_tasks = nullptr;     // MFMA forward: single worldlines of 16 < L < 32 chains
    PackTask* fwdp_tasks = nullptr;
    // the packed tiles of representatives k_dedup lists (P = 2 from the front, P = 4 from
    // n_fwdp2_tasks on; PackTask.p0 indexes prep) and the representatives they hold
    PackTask* fwdpc_tasks = nullptr;
    int32_t* prep = nullptr;
    DrawTask* fwd64_tasks = nullptr;    // MFMA forward: single worldlines of L = 64 chains     // MFMA forward, packed: P = 2 tasks, then P = 4 tasks
    DrawTask* draw32_tasks = nullptr;   // backward: worldline blocks of L = 32 chains
    DrawTask* draww_tasks = nullptr;    // backward, windowed draws (k_backward_win)
    DrawTask* drawx_tasks = nullptr;    // backward: the remaining chains (any L)
    void* ckpt = nullptr;     // FH_FLAG_GRAD_CHECKPOINT: checkpoint and segment rows (plan
                              // precision), in place of the ring rows in the filter workspace
    void* gpart = nullptr;    // matrix-core adjoints: per-group partial field gradients (plan
                              // precision: FP32 for FH_FP32_MFMA3, FP64 for the FP64 circulant)
    void* mala = nullptr;     // fh_mala_field: proposal, two gradients [3][aux_elems] in plan
                              // precision, then log Z_path at both fields [2][n_chains] f64
    double* meas = nullptr;   // fh_measure per-slice rows: S(k) [aux_elems], C(r) [aux_elems],
                              // then the (n_up n_dn, (n_up - n_dn)^2) site sums [slices][2]
    int32_t* perm = nullptr;     // [particles] reconnection at tau = beta: slice L_tau of
                                 // worldline p is slice 0 of worldline perm[part_off + p]
                                 // (chain-local indices); the identity unless changed
    int32_t* perm_inv = nullptr; // [particles] its inverse
    int32_t* sign = nullptr;     // [n_chains] sgn(P_up) sgn(P_dn), +1 or -1
    int32_t* bw_state = nullptr; // backward kernel choice for the windowed chains:
                                 // [0] full-row passes left (0: windowed), [1] current hold
                                 // length, then per chain the uncertified first-window draws
                                 // of the last windowed pass ([kBwCounts + chain])
    int32_t* rescue = nullptr;   // FP32 plans: rescue state words (kRescueFlags), else null
    DrawTask* rescue_list = nullptr;  // blocks queued for the FP64 re-filter, [n_draw_tasks]
    int32_t* rep_slot = nullptr;      // phase A: the slot of each representative's block [blk]
    DrawTask* arep = nullptr;         // phase A: its representatives, densely [n_rescue_slots]
    double* rescue_ws = nullptr;      // [n_rescue_slots][rescue_slot_elems] FP64 filter rows
    double* rescue_w = nullptr;       // [2][aux_elems] FP64 W~ of the chains with queued blocks
    int32_t* status = nullptr;   // [0] first error code, [1] its chain
    uint64_t* sweep = nullptr;   // sweep index read by the kernels
};

}  // namespace fh

struct fh_plan_s {
    int32_t n_chains = 0;
    int32_t precision = 0;
    uint32_t flags = 0;
    std::vector<fh_chain_desc> descs;
    std::vector<fh::ChainInfo> chains;
    std::vector<double> tables;
    std::vector<uint16_t> cmat;
    std::vector<uint16_t> cmatp;
    std::vector<uint16_t> cmatb;
    std::vector<double> cmat64;
    int64_t aux_elems = 0, path_elems = 0, particles = 0, blk_elems = 0, filt_elems = 0;
    int32_t n_fwd_tasks = 0, n_draw_tasks = 0;
    int64_t total_slices = 0;
    int32_t n_groups = 0;
    int32_t n_fwd32_tasks = 0, n_fwdx_tasks = 0, n_draw32_tasks = 0;
    int32_t n_fwdp2_tasks = 0, n_fwdp4_tasks = 0;
    int32_t n_fwd64_tasks = 0;
    int32_t n_fwd64p_tasks = 0;  // 32 < L < 64 on FP32_MFMA3, after the L = 64 tasks in fwd64_tasks
    int32_t max_N_x = 0;  // largest N among the chains of drawx_tasks
    int32_t n_draww_tasks = 0, n_drawx_tasks = 0;
    int32_t n_fwdd_tasks = 0;  // FP64 circulant forward tasks (the FFT takes n_fwd_tasks pairs)
    // after them in fwdd_tasks: the tasks of the 64 x 64, then of the 48 x 48 chains
    int32_t n_fwdd4_tasks = 0, n_fwdd3_tasks = 0;
    bool rescue_l48 = false, rescue_l64 = false;  // FP32 plans: chains the big FP64 re-filter takes
    bool grad_dmfma = false;   // FP64 plan whose chains all have L <= 32: adjoint on the matrix cores
    double win_bound_scale = 1.0;  // test hook: >= 1 inflates every window bound
    bool bw_adapt = true;          // switch clustered chains to the full-row kernels
    int32_t n_full_only_tasks = 0; // backward tasks of chains that never use the window
    int64_t gpart_elems = 0;
    int64_t ckpt_elems = 0;     // FH_FLAG_GRAD_CHECKPOINT: checkpoint + segment rows (elements)
    int32_t n_rescue_slots = 0;     // FP32 plans: wavefronts of k_rescue
    int64_t rescuable_blocks = 0;   // FP32 plans: blocks of the chains the FP64 re-filter takes
    int32_t n_dedup_tasks = 0;      // (chain, spin, block) tasks of k_dedup (chains with dedup)
    bool share_off = false;         // fh_debug_share_filters(plan, 0): every worldline its own rows
    int64_t end_elems = 0;          // end tiles of the chains with dedup (f32 elements)
    int64_t rescue_slot_elems = 0;  // doubles per slot: (B - 1) N of the largest L <= 32 chain
    int64_t total_sites = 0;  // sum of N over the chains
    int32_t max_N = 0, max_L = 0, max_np = 0;
    size_t real_size = 8;
    std::vector<fh::TuneRecord> tune_log;  // FH_FLAG_AUTOTUNE timings, in the order taken
    fh::Device d;
    // state
    bool have_filters = false;
    bool filters_are_ring = false;
    uint64_t last_sweep = 0;
    const int32_t* last_paths = nullptr;
    const void* last_aux = nullptr;  // the field of the last fh_forward_filter (FP64 re-filter)
    void* scratch = nullptr;  // device address of the static scratch array on the plan's device
    // fh_debug_sweep_timing: events recorded around the forward kernels, the backward kernels and
    // the FP64 re-filter of every sweep, and around its phase A on the side stream
    bool timing = false;
    hipEvent_t tev[8] = {};
    // FP32 plans: a sweep re-filters the chains held on FP64 (phase A) on this stream, beside the
    // FP32 forward and backward passes of the other chains on the caller's stream
    hipStream_t side_stream = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // graph cache for fh_sweep
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    void* graph_aux = nullptr;
    int32_t* graph_paths = nullptr;
};

namespace fh {

// The rescue state of a plan as passed to the kernels (all null for FP64 plans).
inline Rescue rescue_args(fh_plan p) {
    Rescue r;
    r.words = p->d.rescue;
    r.flags = p->d.rescue ? p->d.rescue + kRescueChain + kRescuePerChain * p->n_chains : nullptr;
    r.list = p->d.rescue_list;
    r.rep = p->d.rep;
    r.n_chains = p->n_chains;
    return r;
}

// Kernel launchers (fh_kernels.hip / fh_mfma.hip). All enqueue on `s` and return hipError_t.
hipError_t launch_set_sweep(fh_plan p, uint64_t sweep, hipStream_t s);
hipError_t launch_bump_sweep(fh_plan p, hipStream_t s);
hipError_t launch_potentials(fh_plan p, const void* aux, hipStream_t s);
hipError_t launch_forward(fh_plan p, const void* aux, const int32_t* paths, hipStream_t s);
hipError_t launch_forward_dmfma(fh_plan p, const void* aux, const int32_t* paths, hipStream_t s);
hipError_t launch_grad_dmfma(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor,
                             void* grad_aux, hipStream_t s);
hipError_t launch_forward_mfma(fh_plan p, const void* aux, const int32_t* paths, hipStream_t s);
hipError_t launch_logz_reduce(fh_plan p, double* logZ, hipStream_t s);
hipError_t launch_backward(fh_plan p, int32_t* paths, hipStream_t s);
// FP32 plans: clears the rescue queue (before a forward pass), queues whole chains (after it),
// and re-filters (and, with draw, redraws) the queued blocks in FP64. No-ops for FP64 plans.
// Before an FP32 forward pass: the representative map of the shared forward filters.
hipError_t launch_dedup(fh_plan p, const int32_t* paths, hipStream_t s);
// After it: log Z and end-weight floors of the worldlines that share a representative's rows.
hipError_t launch_member_logz(fh_plan p, const int32_t* paths, hipStream_t s);
hipError_t launch_rescue_reset(fh_plan p, hipStream_t s);
hipError_t launch_rescue_expand(fh_plan p, hipStream_t s);  // after the FP32 forward pass
// Before a sweep's FP32 forward pass: queues the held chains whole as phase A.
hipError_t launch_rescue_held(fh_plan p, hipStream_t s);
// The FP64 re-filter of the queue: phase 0 all of it, 1 phase A, 2 the rest (after phase A).
// Phase A runs the representatives' recursions into their slots, then every block's draws from
// its representative's slot (launch_rescue with phase 1).
hipError_t launch_rescue(fh_plan p, const void* aux, int32_t* paths, bool draw, int phase,
                         hipStream_t s);
// Times every radix order of L (k_fft_tune) on stream s and returns the fastest in *best (the
// default order unless another is faster by more than 2%); timings are appended to *log.
hipError_t tune_radix_plan(fh_plan p, int L, const double* tw_dev, hipStream_t s,
                           RadixPlan* best, std::vector<TuneRecord>* log);
hipError_t launch_gibbs(fh_plan p, const int32_t* paths, void* aux, hipStream_t s);
hipError_t launch_local(fh_plan p, const void* aux, int32_t* paths, int n_passes, hipStream_t s);
hipError_t launch_perm_update(fh_plan p, const int32_t* paths, int n_passes, hipStream_t s);
// `work`: 2 aux_elems + 2 total_slices doubles of per-slice rows (the plan's, or the static scratch).
hipError_t launch_measure(fh_plan p, const int32_t* paths, double* Sk, double* Cr, double* D,
                          double* S2, hipStream_t s, double* work);
// Device address of the static scratch array on the current device (taken once per device).
hipError_t scratch_address(void** out);
hipError_t launch_mala_propose(fh_plan p, const void* aux, const void* dlogz, void* prop,
                               double eps, hipStream_t s);
hipError_t launch_mala_accept(fh_plan p, void* aux, const void* prop, const void* g0,
                              const void* g1, const double* logz0, const double* logz1,
                              double eps, int32_t* accepted, hipStream_t s);
hipError_t launch_grad(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor,
                       void* grad_aux, hipStream_t s);
hipError_t launch_grad_reduce(fh_plan p, double* logZ, double* grad_t, hipStream_t s);
// grad_aux = per chain, the sum of its groups' partial slabs in group order (every adjoint).
hipError_t launch_gpart_reduce(fh_plan p, void* grad_aux, hipStream_t s);
// energy[c] <- -(t_c / beta_c) energy[c]: d log Z_path / d t into the kinetic-energy estimate.
hipError_t launch_kinetic_scale(fh_plan p, double* energy, hipStream_t s);
hipError_t launch_grad_mfma(fh_plan p, const void* aux, const int32_t* paths, int32_t anchor,
                            void* grad_aux, hipStream_t s);
hipError_t launch_zero(void* ptr, int64_t bytes, hipStream_t s);
hipError_t launch_scale_copy(float* dst, const float* src, int64_t n, float factor, hipStream_t s);

size_t forward_lds_bytes(fh_plan p);
size_t grad_lds_bytes(fh_plan p);

}  // namespace fh
