// Windowed inverse-CDF draws for backward sampling (Sec. 3.5.2, site form).
//
// The backward step draws r_j from P(r_j = r | r_{j+1} = s) proportional to
//   w_r = max(f_j(r), 0) G(s - r),   G(dx, dy) = g(dx) g(dy),
// as the smallest site r (site order i = x + L y) whose cumulative weight C_r exceeds u C_total.
// g decays factorially with distance (modified Bessel series), so almost all of the weight sits
// in the window Omega of sites within w lattice steps of s in both directions. The draw taken
// on the window alone is provably the full-row draw whenever its two CDF margins exceed a bound
// on the mass outside Omega:
//   * outside mass M_out = sum_{r not in Omega} w_r <= g_out * sum_r max(f_j(r), 0) <= B, with
//     g_out = max_d g(d) * max_{dist(d) > w} g(d) and the row normalised (sum_r f_j(r) = 1 up to
//     rounding; negative FFT round-off is tiny, so kWinMassBound leaves ample room);
//   * let P_q be the window's cumulative weights in site order, tau = u P_last, and q* the first
//     rank with P_q > tau. Every cumulative weight of the full row at a window site is P_q plus
//     some outside mass in [0, M_out], and the full threshold u C_total lies in [tau, tau + B].
//     If P_{q*} - tau > B and tau - P_{q*-1} >= B, every site before q* (inside or outside the
//     window) stays at or below u C_total and site q* exceeds it: the full-row draw is q*.
// Otherwise the draw is retried on the wider window of half-width kWin2W (same certificate with
// its own, far smaller, outside bound), and only then taken over the full row. The first window
// decides nearly every draw of a sampled path; the wider one the draws whose filter mass lies a
// few sites away (strong fields pull the forward filter away from the sampled path). Either way
// the result is the full-row rule's, up to FP64 rounding that a relative allowance of kWinSlack
// covers. The same helpers run in the kernel and in a host mirror.
#pragma once

#include "fh_fft.h"  // FH_HD

namespace fh {

constexpr int kWinMaxW = 3;               // window half-width limit: at most 7 x 7 = 49 sites
constexpr int kWinLanes = 16;             // lanes per worldline in the windowed kernel
constexpr int kWinPerLane = 4;            // window ranks per lane: 16 * 4 >= 49
constexpr int kWinMaxL = 64;              // g(d) for d < L is staged in LDS
constexpr double kWinMassBound = 1.0625;  // >= sum_r max(f_j(r), 0) of a normalised row
constexpr double kWinSlack = 1e-13;       // FP64 rounding allowance, relative to the window mass
constexpr int kWinSelectLog2 = 20;        // w is the smallest with g_out <= 2^-20 max G
constexpr int kWin2W = 7;                 // second window, tried before the full row: 15 x 15

// Window width along one dimension: 2w + 1, or the whole dimension when that covers it.
FH_HD inline int win_width(int w, int L) { return 2 * w + 1 < L ? 2 * w + 1 : L; }

// Coordinates of the window along one dimension, for a window centred on c: the coordinates
// {c - w, ..., c + w} mod L sorted ascending, so that ranks follow site order. When the window
// wraps past 0 or L - 1, the wrapped part comes first (or last). Rank q (0 <= q < WW) sits at
// q when q <= thr and at q + base otherwise (branch-free in the kernel):
//   no wrap:          thr = -1,         base = c - w;
//   wraps below 0:    thr = c + w,      base = L - WW;
//   wraps past L - 1: thr = c + w - L,  base = L - WW;
//   window = whole dimension (WW = L): thr = L.
FH_HD inline void win_axis(int c, int w, int L, int WW, int* thr, int* base) {
    const int lo = c - w, hi = c + w;
    const bool wl = lo < 0, wh = hi >= L;
    *thr = WW == L ? L : wl ? hi : wh ? hi - L : -1;
    *base = (wl || wh) ? L - WW : lo;
}
FH_HD inline int win_at(int q, int thr, int base) { return q + (q <= thr ? 0 : base); }

FH_HD inline int win_coord(int q, int c, int w, int L, int WW) {
    int thr, base;
    win_axis(c, w, L, WW, &thr, &base);
    return win_at(q, thr, base);
}

// The two margin conditions above, with bound = g_out * kWinMassBound + kWinSlack * window mass.
FH_HD inline bool win_certified(double c_lo, double c_hi, double tau, double bound) {
    return (c_hi - tau > bound) && (tau - c_lo >= bound);
}

// Half-width and outside bound for a chain with kernel table g[0..L): the smallest w <= kWinMaxW
// whose window covers the lattice or whose g_out is at most 2^-kWinSelectLog2 max G. Returns
// false (and w = kWinMaxW with its true bound) when none qualifies; the window then still gives
// correct draws, only with frequent fallbacks.
inline bool win_select(const double* g, int L, int* w_out, double* gout_out) {
    double gmax = 0.0;
    for (int d = 0; d < L; ++d) gmax = g[d] > gmax ? g[d] : gmax;
    double gout = 0.0;
    for (int w = 1; w <= kWinMaxW; ++w) {
        gout = 0.0;
        if (win_width(w, L) < L) {
            double m = 0.0;
            for (int d = 0; d < L; ++d) {
                const int dist = d < L - d ? d : L - d;
                if (dist > w && g[d] > m) m = g[d];
            }
            gout = gmax * m;
        }
        *w_out = w;
        *gout_out = gout;
        if (gout <= gmax * gmax * (1.0 / (double)(1 << kWinSelectLog2))) return true;
    }
    return false;
}

// Outside bound of a chain whose half-width w is fixed (after the hopping changes).
inline double win_bound_for(const double* g, int L, int w) {
    if (win_width(w, L) >= L) return 0.0;
    double gmax = 0.0, m = 0.0;
    for (int d = 0; d < L; ++d) {
        gmax = g[d] > gmax ? g[d] : gmax;
        const int dist = d < L - d ? d : L - d;
        if (dist > w && g[d] > m) m = g[d];
    }
    return gmax * m;
}

}  // namespace fh
