// FP64 circulant on the FP64 matrix cores, shared by the FP64 forward filter, the FP64 adjoint
// and the FP64 re-filter of blocks that leave FP32's range (fh_kernels.hip, fh_mfma.hip).
//
// v_mfma_f64_16x16x4_f64 reads A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k, and
// leaves D[i][j] in lane j + 16 (i mod 4), register i / 4 (checked on the device). A 32 x 32
// matrix in that accumulator layout is four 16 x 16 tiles (I, J), tile index 2 I + J; element
// (16 I + 4 r + lane / 16, 16 J + lane % 16) sits in register r of tile (I, J). Register r of
// tile (K, I) is then directly the A operand of X^T with K-index 16 K + 4 r + lane / 16, so
//   (X^T C)(I, J) = sum over K, r of mfma(X(K, I)[r], Cb[(4 K + r) * 2 + J])
// with Cb the matching B operands of the circulant C[k][j] = g((k - j) mod L) (zero outside
// L x L): 32 products per multiplication, no operand splitting, every product and sum in FP64.
// Two multiplications give (F^T C)^T C = C F C, C being symmetric.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace fh {

typedef __attribute__((ext_vector_type(4))) double f64x4;

struct Tile64 {
    f64x4 t[4];
};

__device__ inline Tile64 circ64(const Tile64& X, const double (&Cb)[16]) {
    Tile64 Y;
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
        for (int J = 0; J < 2; ++J) {
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int K = 0; K < 2; ++K)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X.t[2 * K + I][r],
                                                               Cb[(4 * K + r) * 2 + J], acc, 0, 0, 0);
            Y.t[2 * I + J] = acc;
        }
    return Y;
}

// A 64-bit lane exchange by DPP (every lane has its source lane under these controls).
template <int CTRL>
__device__ inline double dpp_swap_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}
__device__ inline double lane_f64(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}
// Sum over the wavefront, the same bits in every lane: each 16-lane row by DPP exchanges (an
// addition and its mirror give the same bits), then the four row sums in one fixed order. No
// LDS round trip (the FP64 recursions wait on this sum every step).
__device__ inline double wave_sum_f64(double v) {
    v += dpp_swap_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_swap_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_swap_f64<0x141>(v);  // row_half_mirror
    v += dpp_swap_f64<0x140>(v);  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Tile coordinates of element (tile q, register r) of a lane: x = 16 (q & 1) + lane % 16,
// y = 16 (q >> 1) + 4 r + lane / 16.
__device__ inline int t64_x(int q, int lane) { return 16 * (q & 1) + (lane & 15); }
__device__ inline int t64_y(int q, int r, int lane) { return 16 * (q >> 1) + 4 * r + (lane >> 4); }

// The forward recursion of one block on the FP64 circulant, one wavefront (Sec. 3.5.2, site
// basis, with the per-step sum normaliser and the log-shifted potentials W~ = W exp(-m_l)):
//   f~_0 = delta_a; h_j = W~_{start+j} . (C f~_{j-1} C); c_j = sum h_j; f~_j = h_j / c_j
//   log Z = la + sum_j (log c_j + m_{start+j}) + log (C f~_{len-1} C)(e),
// where la is log W_start(a), supplied by the caller. wtab(l, w) fills w[4 q + r] with W~ of
// slice l at the lane's element (q, r) (any finite value at padded positions, where C f C is an
// exact zero); put(j, q, r, v) receives element (q, r) of row f~_j, j = 1 .. len - 1, at the
// lane's positions inside the L x L lattice only; put_end(q, r, v) the same elements of the end
// tile C f~_{len-1} C, and *la_end log Z without the end weight (for worldlines that share these
// rows but end elsewhere). Returns log Z; *ok becomes false when a normaliser or the end weight
// is not a positive finite number.
template <typename WTab, typename Put, typename PutEnd>
__device__ inline double dmfma_block_forward_end(const double (&Cb)[16], int L, int L_tau,
                                                 int start, int len, int a, int e, double la,
                                                 const double* __restrict__ shift, WTab wtab,
                                                 Put put, PutEnd put_end, double* la_end,
                                                 bool* ok) {
    const int lane = threadIdx.x & 63;
    auto inside = [&](int q, int r) { return t64_x(q, lane) < L && t64_y(q, r, lane) < L; };
    const int ax = a % L, ay = a / L;
    Tile64 F;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            F.t[q][r] = (t64_x(q, lane) == ax && t64_y(q, r, lane) == ay) ? 1.0 : 0.0;
    bool good = true;
    for (int j = 1; j < len; ++j) {
        const int l = (start + j) % L_tau;
        double w[16];
        wtab(l, w);
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
        good = good && tot > 0.0 && isfinite(tot);
        const double inv = 1.0 / tot;
        la += log(tot) + shift[l];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                F.t[q][r] *= inv;
                if (inside(q, r)) put(j, q, r, F.t[q][r]);
            }
    }
    // end weight (C f~ C)(e)
    const Tile64 H = circ64(circ64(F, Cb), Cb);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (inside(q, r)) put_end(q, r, H.t[q][r]);
    *la_end = la;
    const int ex = e % L, ey = e / L;
    const int qe = 2 * (ey >> 4) + (ex >> 4), re = (ey & 15) >> 2;
    double hv = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (q == qe && r == re) hv = H.t[q][r];
    hv = __shfl(hv, (ex & 15) + 16 * (ey & 3), 64);
    good = good && hv > 0.0;
    *ok = good;
    return la + log(hv);
}

// dmfma_block_forward_end without the end tile.
template <typename WTab, typename Put>
__device__ inline double dmfma_block_forward(const double (&Cb)[16], int L, int L_tau, int start,
                                             int len, int a, int e, double la,
                                             const double* __restrict__ shift, WTab wtab, Put put,
                                             bool* ok) {
    double la_end;
    return dmfma_block_forward_end(Cb, L, L_tau, start, len, a, e, la, shift, wtab, put,
                                   [](int, int, double) {}, &la_end, ok);
}

// Lattices of side L = 16 NT with NT = 3 or 4 (L = 48, 64) on the same instruction. The filter
// is NT x NT tiles of 16 x 16, tile q = NT I + J holding rows 16 I .. and columns 16 J .., its
// element (16 I + 4 r + lane / 16, 16 J + lane % 16) in register r, as above. C[k][j] =
// g((k - j) mod L) is then block-circulant: its 16 x 16 block (K, J) depends only on
// D = (K - J) mod NT, and the B operands are Cb[4 D + r], lane j + 16 k holding
// g((16 D + 4 r + k - j) mod L):
//   (X^T C)(I, J) = sum over K, r of mfma(X(K, I)[r], Cb[4 ((K - J) mod NT) + r]),
// 4 NT^3 products per multiplication, every product and sum in FP64, as for L <= 32.
template <int NT>
struct TileBig {
    f64x4 t[NT * NT];
};

template <int NT>
__device__ inline void circ_big(const TileBig<NT>& X, const double (&Cb)[16], TileBig<NT>& Y) {
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = 0; J < NT; ++J) {
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int K = 0; K < NT; ++K)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        X.t[NT * K + I][r], Cb[4 * ((K - J + NT) % NT) + r], acc, 0, 0, 0);
            Y.t[NT * I + J] = acc;
        }
}

// Site coordinates of element (tile q, register r) of a lane in the NT x NT tiling.
template <int NT>
__device__ inline int tb_x(int q, int lane) { return 16 * (q % NT) + (lane & 15); }
template <int NT>
__device__ inline int tb_y(int q, int r, int lane) { return 16 * (q / NT) + 4 * r + (lane >> 4); }

// dmfma_block_forward_end for L = 16 NT: the same recursion, normaliser, log Z and outputs.
// wtab(l, w) fills w[4 q + r] with W~ of slice l at the lane's element (q, r); every element is
// a lattice site, so put and put_end see all of them.
template <int NT, typename WTab, typename Put, typename PutEnd>
__device__ inline double dmfma_big_block_forward_end(const double (&Cb)[16], int L_tau,
                                                     int start, int len, int a, int e, double la,
                                                     const double* __restrict__ shift, WTab wtab,
                                                     Put put, PutEnd put_end, double* la_end,
                                                     bool* ok) {
    constexpr int L = 16 * NT, NQ = NT * NT;
    const int lane = threadIdx.x & 63;
    const int ax = a % L, ay = a / L;
    TileBig<NT> F, X;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            F.t[q][r] = (tb_x<NT>(q, lane) == ax && tb_y<NT>(q, r, lane) == ay) ? 1.0 : 0.0;
    bool good = true;
    for (int j = 1; j < len; ++j) {
        const int l = (start + j) % L_tau;
        circ_big<NT>(F, Cb, X);
        circ_big<NT>(X, Cb, F);
        // W after the products: loaded before them, the slice would need 2 NT^2 more registers
        double w[4 * NQ];
        wtab(l, w);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                F.t[q][r] *= w[4 * q + r];
                sum += F.t[q][r];
            }
        const double tot = wave_sum_f64(sum);
        good = good && tot > 0.0 && isfinite(tot);
        const double inv = 1.0 / tot;
        la += log(tot) + shift[l];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                F.t[q][r] *= inv;
                put(j, q, r, F.t[q][r]);
            }
    }
    // end weight (C f~ C)(e)
    circ_big<NT>(F, Cb, X);
    circ_big<NT>(X, Cb, F);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) put_end(q, r, F.t[q][r]);
    *la_end = la;
    const int ex = e % L, ey = e / L;
    const int qe = NT * (ey >> 4) + (ex >> 4), re = (ey & 15) >> 2;
    double hv = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (q == qe && r == re) hv = F.t[q][r];
    hv = __shfl(hv, (ex & 15) + 16 * (ey & 3), 64);
    good = good && hv > 0.0;
    *ok = good;
    return la + log(hv);
}

}  // namespace fh
