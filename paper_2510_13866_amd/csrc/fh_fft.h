// Mixed-radix (2, 3, 4) Stockham FFT stages for L x L complex tiles.
//
// The same stage code runs inside the GPU kernels (one butterfly per thread, LDS ping-pong
// buffers) and in a host self-test (a loop over butterflies), so the index arithmetic is checked
// on the CPU before any launch. Forward transform: X(k) = sum_n x(n) exp(-2 pi i k n / L) per
// dimension; the inverse uses the conjugate twiddles and is NOT scaled (callers fold 1/N into
// the spectral multiplier).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define FH_HD __host__ __device__
#else
#define FH_HD
#endif

namespace fh {

template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
FH_HD inline cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
FH_HD inline cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
FH_HD inline cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
FH_HD inline cpx<T> rot90(cpx<T> a) {
    return INV ? cpx<T>{-a.im, a.re} : cpx<T>{a.im, -a.re};
}

constexpr int kMaxRadices = 6;
constexpr int kMaxL = 64;

// Radix plan of one dimension: L = prod rad[0..n).
struct RadixPlan {
    int32_t n;
    int32_t rad[kMaxRadices];
};

// Default factorisation: radix-4 stages, then one radix-2 if needed, then radix-3 stages.
// Returns false when L is not of the form 2^a 3^b or too long.
inline bool default_radix_plan(int L, RadixPlan* p) {
    p->n = 0;
    int r = L;
    while (r % 4 == 0 && p->n < kMaxRadices) { p->rad[p->n++] = 4; r /= 4; }
    if (r % 2 == 0 && p->n < kMaxRadices) { p->rad[p->n++] = 2; r /= 2; }
    while (r % 3 == 0 && p->n < kMaxRadices) { p->rad[p->n++] = 3; r /= 3; }
    return r == 1 && L >= 2 && L <= kMaxL;
}

// Every ordered sequence of radices from {2, 3, 4} with product L and at most kMaxRadices
// stages, each exactly once (a depth-first walk over the radix of the next stage). These are the
// candidates the autotuner times. Writes min(count, cap) plans to out; returns the count.
inline int radix_orders(int L, RadixPlan* out, int cap) {
    struct Walk {
        RadixPlan* out;
        int cap, count;
        RadixPlan cur;
        void go(int rest) {
            if (rest == 1) {
                if (cur.n > 0) {
                    if (count < cap) out[count] = cur;
                    ++count;
                }
                return;
            }
            if (cur.n == kMaxRadices) return;
            const int radices[3] = {4, 2, 3};
            for (int r : radices)
                if (rest % r == 0) {
                    cur.rad[cur.n++] = r;
                    go(rest / r);
                    --cur.n;
                }
        }
    };
    if (L < 2 || L > kMaxL) return 0;
    Walk w{out, cap, 0, {}};
    w.cur.n = 0;
    for (int i = 0; i < kMaxRadices; ++i) w.cur.rad[i] = 0;
    w.go(L);
    return w.count;
}

// A plan is usable when its radices are in {2, 3, 4}, there are 1..kMaxRadices of them and
// their product is L.
inline bool valid_radix_plan(int L, const RadixPlan& p) {
    if (p.n < 1 || p.n > kMaxRadices || L < 2 || L > kMaxL) return false;
    int prod = 1;
    for (int i = 0; i < p.n; ++i) {
        if (p.rad[i] != 2 && p.rad[i] != 3 && p.rad[i] != 4) return false;
        prod *= p.rad[i];
    }
    return prod == L;
}

// One small DFT of length P in {2, 3, 4}, in place on v.
template <typename T, bool INV, int P>
FH_HD inline void small_dft(cpx<T>* v) {
    if (P == 2) {
        cpx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (P == 4) {
        cpx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        cpx<T> c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        cpx<T> rd = rot90<T, INV>(d);
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, rd);
        v[3] = csub(b, rd);
    } else {  // P == 3
        const T h = T(0.86602540378443864676);  // sqrt(3)/2
        cpx<T> s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        cpx<T> m = {v[0].re - T(0.5) * s.re, v[0].im - T(0.5) * s.im};
        cpx<T> rd = rot90<T, INV>(cpx<T>{h * d.re, h * d.im});  // -+ i h d
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, rd);
        v[2] = csub(m, rd);
    }
}

// Butterfly b (0 <= b < L*(L/P)) of one Stockham stage along one dimension of an L x L tile.
// line_stride / elem_stride select the dimension: rows (L, 1) or columns (1, L).
// Ns = product of the radices of the earlier stages of this dimension.
// tw[m] = exp(-2 pi i m / L), m in [0, L).
template <typename T, bool INV, int P>
FH_HD inline void stockham_butterfly(int b, int L, int Ns, int line_stride, int elem_stride,
                                     const cpx<T>* src, cpx<T>* dst, const cpx<T>* tw) {
    const int per_line = L / P;
    const int line = b / per_line;
    const int j = b - line * per_line;
    const int base = line * line_stride;
    const int k = j % Ns;
    cpx<T> v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = src[base + (j + q * per_line) * elem_stride];
    if (Ns > 1) {
        const int step = L / (Ns * P);
#pragma unroll
        for (int q = 1; q < P; ++q) {
            cpx<T> w = tw[(q * k * step) % L];
            if (INV) w.im = -w.im;
            v[q] = cmul(v[q], w);
        }
    }
    small_dft<T, INV, P>(v);
    const int out0 = (j / Ns) * Ns * P + k;
#pragma unroll
    for (int q = 0; q < P; ++q) dst[base + (out0 + q * Ns) * elem_stride] = v[q];
}

// Runtime radix dispatch.
template <typename T, bool INV>
FH_HD inline void stockham_butterfly_rt(int p, int b, int L, int Ns, int line_stride,
                                        int elem_stride, const cpx<T>* src, cpx<T>* dst,
                                        const cpx<T>* tw) {
    if (p == 4)
        stockham_butterfly<T, INV, 4>(b, L, Ns, line_stride, elem_stride, src, dst, tw);
    else if (p == 2)
        stockham_butterfly<T, INV, 2>(b, L, Ns, line_stride, elem_stride, src, dst, tw);
    else
        stockham_butterfly<T, INV, 3>(b, L, Ns, line_stride, elem_stride, src, dst, tw);
}

}  // namespace fh
