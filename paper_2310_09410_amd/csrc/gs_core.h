// Rank-revealing projection of one subsystem (device code shared by the
// plain and the batched precompute). See gs_project.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ldopf {

__device__ inline double gs_wave_sum(double v) {
    // xor butterfly: every lane ends with the same bits (addition commutes)
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// One wave, one subsystem of n <= 64 NQ variables (lane l owns columns l,
// l + 64, ..., in registers). Row i of A_s is As[i * n + c]; when fscale is
// given, a row carrying load row_load[i] has its right-hand side and its
// coefficient in column row_wcol[i] multiplied by fscale[row_load[i]] (the
// load scaling of a scenario). Writes the basis U (n x n), bbar (n) and, when
// abar is not null, the dense Abar (n x n); returns the rank and sets *bad
// when a dependent row has an inconsistent right-hand side.
template <int NQ>
__device__ inline int gs_project(int lane, int n, int m, const double* As, const double* bs, const int32_t* rload,
                          const int32_t* rwcol, const double* fscale, double tol_dep, double tol_rhs, double* U,
                          double* beta, double* bb, double* Ab, int* bad_out) {
    auto scale_of = [&](int i) -> double {
        if (!fscale) return 1.0;
        const int l = rload[i];
        return l >= 0 ? fscale[l] : 1.0;
    };
    auto coef = [&](int i, int c) -> double {
        const double v = As[int64_t(i) * n + c];
        if (!fscale) return v;
        return (c == rwcol[i]) ? v * scale_of(i) : v;
    };
    double bmax = 0.0;
    for (int i = 0; i < m; ++i) bmax = fmax(bmax, fabs(bs[i] * scale_of(i)));
    int r = 0, bad = 0;
    for (int i = 0; i < m; ++i) {
        double ar[NQ];
        double nn = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = lane + 64 * q;
            ar[q] = c < n ? coef(i, c) : 0.0;
            nn += ar[q] * ar[q];
        }
        const double nrm0 = sqrt(gs_wave_sum(nn));
        double bi = bs[i] * scale_of(i);
        for (int pass = 0; pass < 2; ++pass) {
            for (int k = 0; k < r; ++k) {
                double d = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int c = lane + 64 * q;
                    if (c < n) d += ar[q] * U[int64_t(k) * n + c];
                }
                d = gs_wave_sum(d);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int c = lane + 64 * q;
                    if (c < n) ar[q] -= d * U[int64_t(k) * n + c];
                }
                bi -= d * beta[k];
            }
        }
        nn = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) nn += ar[q] * ar[q];
        const double nr = sqrt(gs_wave_sum(nn));
        if (nrm0 > 0.0 && nr > tol_dep * nrm0 && r < n) {
            const double inv = 1.0 / nr;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int c = lane + 64 * q;
                if (c < n) U[int64_t(r) * n + c] = ar[q] * inv;
            }
            if (lane == 0) beta[r] = bi * inv;
            ++r;
        } else if (fabs(bi) > tol_rhs * (1.0 + bmax)) {
            bad = 1;  // dependent row with an inconsistent right-hand side
        }
    }
    // complete the basis: greedily take the unit vector farthest from the span
    for (int q2 = r; q2 < n; ++q2) {
        double best = -1.0;
        int bidx = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = lane + 64 * q;
            if (c < n) {
                double res = 1.0;
                for (int k = 0; k < q2; ++k) {
                    const double u = U[int64_t(k) * n + c];
                    res -= u * u;
                }
                if (res > best) { best = res; bidx = c; }
            }
        }
        for (int mm = 32; mm >= 1; mm >>= 1) {
            const double ob = __shfl_xor(best, mm, 64);
            const int oi = __shfl_xor(bidx, mm, 64);
            if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
        }
        double ar[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) ar[q] = (lane + 64 * q) == bidx ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int k = 0; k < q2; ++k) {
                double d = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int c = lane + 64 * q;
                    if (c < n) d += ar[q] * U[int64_t(k) * n + c];
                }
                d = gs_wave_sum(d);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int c = lane + 64 * q;
                    if (c < n) ar[q] -= d * U[int64_t(k) * n + c];
                }
            }
        }
        double nn = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) nn += ar[q] * ar[q];
        const double inv = 1.0 / sqrt(gs_wave_sum(nn));
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = lane + 64 * q;
            if (c < n) U[int64_t(q2) * n + c] = ar[q] * inv;
        }
    }
    // bbar = Q' beta over the row-space rows
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int c = lane + 64 * q;
        if (c < n) {
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc += beta[k] * U[int64_t(k) * n + c];
            bb[c] = acc;
        }
    }
    // dense Abar = Q'Q - I; entry (i, c) needs column i, owned by lane i % 64
    for (int i = 0; Ab && i < n; ++i) {
        const int owner = i & 63;
        double acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
        for (int k = 0; k < r; ++k) {
            const double mine = lane == owner ? U[int64_t(k) * n + i] : 0.0;
            const double ui = __shfl(mine, owner, 64);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int c = lane + 64 * q;
                if (c < n) acc[q] += ui * U[int64_t(k) * n + c];
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = lane + 64 * q;
            if (c < n) Ab[int64_t(i) * n + c] = acc[q] - (c == i ? 1.0 : 0.0);
        }
    }
    *bad_out = bad;
    return r;
}

}  // namespace ldopf
