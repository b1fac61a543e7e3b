// Streamed sweep: the path for problems whose operators and state do not fit
// the LDS of one workgroup per CU (the persistent sweep's requirement).
//
// The same sweep as the persistent kernel (Algorithm 1: global update of
// closed_1 in its derived form, local update of closed_2 in rank form, dual
// update ADMM-3, the residual sums and the test of Section III-C), with every
// operand in HBM and one launch per sweep: a wave takes a group of
// subsystems, a lane a row, and forms the global update of that row's
// variable from the previous sweep's copies (closed_1: their x_s and lambda
// over a padded table of the first four copies and a CSR list), then t_k =
// sum_j W_kj v_j by a sum over the subsystem's lanes, y_j = bbar_j + v_j -
// sum_k W_kj t_k in mode 1 or bbar_j + sum_k W_kj t_k in mode 0 (W the K_s
// rows of the precomputed basis that span the smaller of the row space and
// its complement), the dual update and the residual sums of its block. Block 0
// of each launch instead runs the test of Section III-C on the previous
// launch's block sums, in a fixed order, and stops the solve or numbers the
// sweep. Sweep k reads x_s and lambda of sweep k - 1 and writes its own into
// the other of two buffers (sweep k in buffer k % 2), its block sums and x
// likewise, so a launch never reads what it writes, and the state of the
// sweep that passed the test survives the launch that runs beside the test.
// A launch after the stop returns at once, so C sweeps are captured in one
// HIP graph and the host replays it until the test holds. FP64 throughout;
// the returned state is that of the sweep that passed the test.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "problem.h"

namespace ldopf {

namespace {

constexpr int kSWaves = 4;    // waves per block
constexpr int kSBlocks = 2048; // blocks of subsystem groups per launch: rows of partial sums
constexpr int kSGraph = 32;   // sweeps per captured graph
constexpr int kGroupWords = 20;  // words per group record

struct StreamArgs {
    int64_t S, n, nloc;
    // per group of subsystems (kGroupWords words): lanes each, count, largest
    // K_s, 0, then per slot (up to 4) n_s | K_s << 12 | mode << 24, its first
    // copy, and the offset of its K_s rows in the basis (two words)
    const int32_t* groups;
    int64_t n_groups;
    const int32_t* gidx;
    const int32_t* var_off;
    const int32_t* var_copy;
    const int4* ell;  // per variable its first four copies, -1 padded
    const double* basis;
    const double* bbar;
    const double4* vconst;  // per variable: c, lower bound, upper bound, copy count
    double* x;              // the half of the two-part x buffer this sweep writes
    const double* u_rd;     // u = x_s - lambda / rho and lambda of the previous sweep
    const double* lam_rd;
    double* u_wr;           // u and lambda of this sweep (sweep k in buffer k % 2)
    double* lam_wr;
    const double* part_rd;  // block sums of the previous sweep [kSBlocks][5], tested here
    double* part_wr;        // block sums of this sweep
    int64_t* ctrl; // [0] the sweep being computed (tested by the next launch), [1] stopped
    double* hist;
    int64_t hist_cap;
    SweepStatus* st;
    double rho, eps_rel, eps_abs;
    int64_t max_iter;
    int32_t check;
};

// DPP lane moves inside each row of 16 lanes (gfx9 encodings): quad_perm
// [1,0,3,2] swaps neighbours, quad_perm [2,3,0,1] swaps pairs,
// row_half_mirror reverses each group of 8, row_mirror each row of 16.
template <int CTRL>
__device__ inline double row_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sums of kKB values over aligned groups of G lanes (G = 16, 32 or 64), the
// kKB chains side by side; every lane of a group ends with the same bits:
// within each row of 16 by DPP moves, across rows by lane exchanges. Every
// lane of the wave must be active.
template <int N>
__device__ inline void group_sums(double (&t)[N], int G) {
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] += row_move<0xB1>(t[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] += row_move<0x4E>(t[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] += row_move<0x141>(t[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] += row_move<0x140>(t[i]);
    if (G >= 32)
#pragma unroll
        for (int i = 0; i < N; ++i) t[i] += __shfl_xor(t[i], 16, 64);
    if (G >= 64)
#pragma unroll
        for (int i = 0; i < N; ++i) t[i] += __shfl_xor(t[i], 32, 64);
}

__global__ void stream_init_kernel(StreamArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    a.ctrl[0] = 0;
    a.ctrl[1] = a.max_iter == 0 ? 1 : 0;
    SweepStatus* st = a.st;
    st->iters = 0;
    st->computed = 0;
    st->converged = 0;
    st->flags = 0;
    st->pres = st->dres = st->eps_p = st->eps_d = 0.0;
    st->rho = a.rho;
    st->rho_changes = 0;
}

// Block 0 of a launch: the test of the sweep the previous launch computed
// (its blocks' residual rows in a fixed order: thread r takes rows r,
// r + 64 kSWaves, ..., then sums over each wave and the waves in order), its
// history row and status; then either the stop or the next sweep's number.
// Every thread of the block calls it.
__device__ void stream_test(const StreamArgs& a, int rows) {
    __shared__ double red[kSWaves][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = a.ctrl[0];
    if (t >= 1) {
        double p[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int r = threadIdx.x; r < rows; r += 64 * kSWaves)
#pragma unroll
            for (int q = 0; q < 5; ++q) p[q] += a.part_rd[int64_t(r) * 5 + q];
        group_sums(p, 64);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 5; ++q) red[wv][q] = p[q];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (t < 1) {
        a.ctrl[0] = 1;
        return;
    }
    double d[5];
    for (int q = 0; q < 5; ++q) {
        d[q] = 0.0;
        for (int w = 0; w < kSWaves; ++w) d[q] += red[w][q];
    }
    const double sq = sqrt(double(a.nloc));
    const double pres = sqrt(d[0]), dres = a.rho * sqrt(d[1]);
    const double eps_p = sq * a.eps_abs + a.eps_rel * fmax(sqrt(d[2]), sqrt(d[3]));
    const double eps_d = sq * a.eps_abs + a.eps_rel * sqrt(d[4]);
    if (t <= a.hist_cap) {
        double* h = a.hist + (t - 1) * 4;
        h[0] = pres;
        h[1] = dres;
        h[2] = eps_p;
        h[3] = eps_d;
    }
    const bool conv = pres <= eps_p && dres <= eps_d;
    const bool bad = !isfinite(d[0] + d[1] + d[2] + d[3] + d[4]);
    SweepStatus* st = a.st;
    st->iters = t;
    st->computed = t;
    st->converged = conv ? 1 : 0;
    st->pres = pres;
    st->dres = dres;
    st->eps_p = eps_p;
    st->eps_d = eps_d;
    if (bad) st->flags |= 2;
    if (bad || (a.check && conv) || t >= a.max_iter)
        a.ctrl[1] = 1;
    else
        a.ctrl[0] = t + 1;
}

// closed_1 for variable v: x_v = clip((sum_c u_c - c_v / rho) / N_v) over
// the copies c of v in the previous sweep, u = x_s - lambda / rho, in copy
// order (a NaN passes the clip); the first four copies come from a padded
// table, so that their loads are in flight together, further ones from the
// CSR list.
__device__ inline double global_x(const StreamArgs& a, int v, int* first) {
    const int4 e = a.ell[v];
    *first = e.x;
    const int q0 = a.var_off[v], q1 = a.var_off[v + 1];
    const int ec[4] = {e.x, e.y, e.z, e.w};
    double u4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) u4[i] = ec[i] >= 0 ? a.u_rd[ec[i]] : 0.0;
    double su = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (q0 + i < q1) su += u4[i];
    for (int q = q0 + 4; q < q1; ++q) su += a.u_rd[a.var_copy[q]];
    const double4 k = a.vconst[v];
    const double xh = (su - k.x / a.rho) / k.w;
    return xh < k.y ? k.y : (xh > k.z ? k.z : xh);
}

// u = x_s - lambda / rho of every copy, before the first sweep (from the
// handle's x_s and lambda: the initial point or a warm start)
__global__ void stream_u_kernel(StreamArgs a, const double* xs, const double* lam) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c < a.nloc) a.u_wr[c] = xs[c] - lam[c] * (1.0 / a.rho);
}

// x_s = u + lambda / rho of the returned sweep, into the handle's x_s
__global__ void stream_xs_kernel(StreamArgs a, double* xs) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c < a.nloc) xs[c] = a.u_rd[c] + a.lam_rd[c] * (1.0 / a.rho);
}

// One sweep: closed_1 for each row's variable, closed_2, ADMM-3 and the
// residual sums. A wave takes one group of subsystems at a time: four of at
// most 16 variables (16 lanes each), two of at most 32, or one (64 lanes, NQ
// rows per lane, n_s <= 64 NQ); a lane holds row j of its subsystem, forms
// x of the row's variable (each copy's lane forms the same bits; the lane of
// the variable's first copy writes them), and t_k is a sum over the
// subsystem's lanes. Operator rows are
// loaded kKB at a time (fewer for more rows per lane, so that the batch
// stays in registers). Block 0 runs the test of the previous sweep instead;
// a block that sees the stop it decides skips its groups, which only spares
// buffers the returned sweep does not use.
template <int NQ>
__global__ __launch_bounds__(64 * kSWaves) void stream_sweep_kernel(StreamArgs a, int rows) {
    constexpr int kKB = NQ >= 16 ? 1 : 2;
    if (a.ctrl[1]) return;
    if (blockIdx.x == 0) {
        stream_test(a, rows);
        return;
    }
    __shared__ double red[kSWaves][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t blk = int64_t(blockIdx.x) - 1, nblk = int64_t(gridDim.x) - 1;
    const double rho = a.rho, irho = 1.0 / a.rho;
    double p[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t g = blk * kSWaves + __builtin_amdgcn_readfirstlane(wv); g < a.n_groups; g += nblk * kSWaves) {
        // the group record is the same for the whole wave (scalar loads); a
        // lane takes its slot's words from it
        const int32_t* gr = a.groups + kGroupWords * g;
        const int G = gr[0], count = gr[1], kmax = gr[2];
        const int slot = lane / G, jl = lane - slot * G;
        int nkm = 0, r0 = 0, wlo = 0, whi = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (slot == i && i < count) {
                nkm = gr[4 + 4 * i];
                r0 = gr[5 + 4 * i];
                wlo = gr[6 + 4 * i];
                whi = gr[7 + 4 * i];
            }
        const int n = nkm & 0xfff, K = (nkm >> 12) & 0xfff, mode = (nkm >> 24) & 1;
        const int64_t row0 = r0;
        const double* W = a.basis + ((int64_t(whi) << 32) | uint32_t(wlo));
        double z[NQ], l[NQ], xo[NQ], v[NQ], acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = jl + 64 * q;
            z[q] = l[q] = xo[q] = v[q] = acc[q] = 0.0;
            if (j < n) {
                const int64_t c = row0 + j;
                const int var = a.gidx[c];
                int first;
                z[q] = global_x(a, var, &first);
                if (first == c) a.x[var] = z[q];  // written once, by the variable's first copy
                l[q] = a.lam_rd[c];
                xo[q] = a.u_rd[c] + l[q] * irho;  // x_s of the previous sweep
                v[q] = z[q] + l[q] * irho;
            }
        }
        if constexpr (NQ == 1) {
            // one row per lane: batches of kKB operator rows, the next batch
            // issued before the current one is used. Rows past K_s or lanes
            // past n_s read an address inside the operator (or the first
            // basis word, for an idle lane or K_s = 0) and contribute zero:
            // v is zero past n_s and t_k is masked past K_s, so every load
            // is unconditional
            const int Kc = K > 0 ? K : 1, nc = n > 0 ? n : 1;
            const double* Wl = K > 0 ? W : a.basis;
            const int jc = jl < nc ? jl : nc - 1;
            auto issue = [&](double (&w)[kKB], int k0) {
#pragma unroll
                for (int kb = 0; kb < kKB; ++kb) {
                    const int k = k0 + kb < Kc ? k0 + kb : Kc - 1;
                    w[kb] = Wl[int64_t(k) * nc + jc];
                }
            };
            auto use = [&](const double (&w)[kKB], int k0) {
                double t[kKB];
#pragma unroll
                for (int kb = 0; kb < kKB; ++kb) t[kb] = w[kb] * v[0];
                group_sums(t, G);
#pragma unroll
                for (int kb = 0; kb < kKB; ++kb) acc[0] += w[kb] * (k0 + kb < K ? t[kb] : 0.0);
            };
            double wa[kKB], wb[kKB];
            issue(wa, 0);
            for (int k0 = 0;; k0 += 2 * kKB) {
                issue(wb, k0 + kKB);
                use(wa, k0);
                if (k0 + kKB >= kmax) break;
                issue(wa, k0 + 2 * kKB);
                use(wb, k0 + kKB);
                if (k0 + 2 * kKB >= kmax) break;
            }
        } else
        // all loads of a batch first, then its lane-group sums side by side
        for (int k0 = 0; k0 < kmax; k0 += kKB) {
            double w[kKB][NQ];
#pragma unroll
            for (int kb = 0; kb < kKB; ++kb)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int j = jl + 64 * q;
                    w[kb][q] = (j < n && k0 + kb < K) ? W[int64_t(k0 + kb) * n + j] : 0.0;
                }
            double t[kKB];
#pragma unroll
            for (int kb = 0; kb < kKB; ++kb) {
                t[kb] = 0.0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) t[kb] += w[kb][q] * v[q];
            }
            group_sums(t, G);
#pragma unroll
            for (int kb = 0; kb < kKB; ++kb)
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[q] += w[kb][q] * t[kb];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = jl + 64 * q;
            if (j < n) {
                const int64_t c = row0 + j;
                const double y = a.bbar[c] + (mode ? v[q] - acc[q] : acc[q]);
                const double l1 = l[q] + rho * (z[q] - y);
                a.u_wr[c] = y - l1 * irho;
                a.lam_wr[c] = l1;
                const double dz = z[q] - y, dx = y - xo[q];
                p[0] += dz * dz;
                p[1] += dx * dx;
                p[2] += z[q] * z[q];
                p[3] += y * y;
                p[4] += l1 * l1;
            }
        }
    }
    // the wave's sums, then the waves in order
    group_sums(p, 64);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 5; ++q) red[wv][q] = p[q];
    __syncthreads();
    if (threadIdx.x < 5) {
        double t = 0.0;
        for (int w = 0; w < kSWaves; ++w) t += red[w][threadIdx.x];
        a.part_wr[blk * 5 + threadIdx.x] = t;
    }
}

StreamArgs stream_args(ldopf_problem& h) {
    StreamArgs a{};
    a.S = h.lp.S;
    a.n = h.lp.n;
    a.nloc = int64_t(h.lp.gidx.size());
    a.groups = h.s_groups.p;
    a.n_groups = h.s_n_groups;
    a.gidx = h.s_gidx.p;
    a.var_off = h.s_var_off.p;
    a.var_copy = h.s_var_copy.p;
    a.ell = h.s_ell.p;
    a.basis = h.basis.p;
    a.bbar = h.bbar.p;
    a.vconst = h.s_vconst.p;
    // sweep k reads buffer (k - 1) % 2 and writes buffer k % 2; lambda's
    // buffer 0 is the handle's lambda, u's is filled from the handle's x_s
    // and lambda (the initial point or a warm start) before the first sweep
    a.x = h.s_x2.p;
    a.u_rd = h.s_u2.p;
    a.lam_rd = h.lam.p;
    a.u_wr = h.s_u2.p + h.lp.gidx.size();
    a.lam_wr = h.s_lam2.p;
    a.part_rd = h.s_part.p;
    a.part_wr = h.s_part.p + size_t(kSBlocks) * 5;
    a.ctrl = h.s_ctrl.p;
    a.hist = h.hist.p;
    a.hist_cap = h.opts.history ? int64_t(h.hist.count / 4) : 0;
    a.st = h.st.p;
    a.rho = h.opts.rho;
    a.eps_rel = h.opts.eps_rel;
    a.eps_abs = h.opts.eps_abs;
    a.max_iter = h.opts.max_iter;
    a.check = h.opts.check_termination;
    return a;
}

const void* sweep_kernel_for(int nq) {
    switch (nq) {
        case 1: return reinterpret_cast<const void*>(&stream_sweep_kernel<1>);
        case 4: return reinterpret_cast<const void*>(&stream_sweep_kernel<4>);
        default: return reinterpret_cast<const void*>(&stream_sweep_kernel<16>);
    }
}

void drop_stream_graph(ldopf_problem& h) {
    if (h.s_exec) {
        (void)hipGraphExecDestroy(h.s_exec);
        h.s_exec = nullptr;
    }
    if (h.s_graph) {
        (void)hipGraphDestroy(h.s_graph);
        h.s_graph = nullptr;
    }
}

}  // namespace

void stream_prepare(ldopf_problem& h) {
    const ConsensusLP& lp = h.lp;
    hipStream_t s = h.stream;
    const int64_t S = lp.S, nloc = int64_t(lp.gidx.size());
    if (nloc >= (int64_t(1) << 31) || lp.n >= (int64_t(1) << 31))
        fail(LDOPF_UNSUPPORTED, "the streamed sweep indexes copies and variables with 32-bit integers");
    std::vector<int64_t> meta(size_t(3) * S);
    int64_t off = 0, rank_words = 0;
    int32_t max_n = 1;
    for (int64_t i = 0; i < S; ++i) {
        const int64_t n = lp.ns[i], r = h.rank[i];
        const int64_t mode = r <= n - r ? 1 : 0, K = std::min(r, n - r);
        meta[3 * i] = n | (K << 16) | (mode << 32);
        meta[3 * i + 1] = lp.loc_off[i];
        meta[3 * i + 2] = off + (mode ? 0 : r) * n;  // the K rows of the basis that the rank form uses
        off += n * n;
        rank_words += n * K;
        max_n = std::max<int32_t>(max_n, int32_t(n));
    }
    std::vector<int32_t> g32(nloc), var_off(lp.n + 1, 0), var_copy(nloc);
    for (int64_t c = 0; c < nloc; ++c) {
        g32[c] = int32_t(lp.gidx[c]);
        var_off[lp.gidx[c] + 1]++;
    }
    for (int64_t v = 0; v < lp.n; ++v) var_off[v + 1] += var_off[v];
    std::vector<int32_t> fill(var_off.begin(), var_off.end() - 1);
    for (int64_t c = 0; c < nloc; ++c) var_copy[fill[lp.gidx[c]]++] = int32_t(c);
    // groups of subsystems per wave: the largest first (longest chains),
    // then pairs of at most 32 variables, then fours of at most 16; with any
    // subsystem above 64 variables, one subsystem per wave throughout
    std::vector<int32_t> groups;
    int64_t n_groups = 0;
    auto add_group = [&](int32_t G, const std::vector<int32_t>& subs) {
        int32_t kmax = 0;
        for (int32_t q : subs) kmax = std::max<int32_t>(kmax, int32_t((meta[3 * size_t(q)] >> 16) & 0xffff));
        const size_t at = groups.size();
        groups.resize(at + kGroupWords, 0);
        groups[at] = G;
        groups[at + 1] = int32_t(subs.size());
        groups[at + 2] = kmax;
        for (size_t i = 0; i < subs.size(); ++i) {
            const int64_t q = subs[i], m0 = meta[3 * size_t(q)];
            const int64_t n = m0 & 0xffff, K = (m0 >> 16) & 0xffff, mode = (m0 >> 32) & 1;
            const int64_t woff = meta[3 * size_t(q) + 2];
            groups[at + 4 + 4 * i] = int32_t(n | (K << 12) | (mode << 24));
            groups[at + 5 + 4 * i] = int32_t(meta[3 * size_t(q) + 1]);
            groups[at + 6 + 4 * i] = int32_t(uint32_t(uint64_t(woff) & 0xffffffffu));
            groups[at + 7 + 4 * i] = int32_t(uint32_t(uint64_t(woff) >> 32));
        }
        ++n_groups;
    };
    std::vector<int32_t> s16, s32, s64;
    for (int64_t i = 0; i < S; ++i) {
        const int32_t n = lp.ns[i];
        if (max_n > 64 || n > 32) s64.push_back(int32_t(i));
        else if (n > 16) s32.push_back(int32_t(i));
        else s16.push_back(int32_t(i));
    }
    for (int32_t q : s64) add_group(64, {q});
    for (size_t i = 0; i < s32.size(); i += 2)
        add_group(32, std::vector<int32_t>(s32.begin() + i, s32.begin() + std::min(s32.size(), i + 2)));
    for (size_t i = 0; i < s16.size(); i += 4)
        add_group(16, std::vector<int32_t>(s16.begin() + i, s16.begin() + std::min(s16.size(), i + 4)));
    h.s_groups.upload(groups, s, "upload streamed plan");
    h.s_n_groups = n_groups;
    h.s_gidx.upload(g32, s, "upload streamed plan");
    h.s_var_off.upload(var_off, s, "upload streamed plan");
    h.s_var_copy.upload(var_copy, s, "upload streamed plan");
    std::vector<int4> ell(lp.n);
    for (int64_t v = 0; v < lp.n; ++v) {
        int32_t e[4] = {-1, -1, -1, -1};
        for (int32_t i = 0; i < 4 && var_off[v] + i < var_off[v + 1]; ++i) e[i] = var_copy[var_off[v] + i];
        ell[v] = int4{e[0], e[1], e[2], e[3]};
    }
    h.s_ell.upload(ell, s, "upload streamed plan");
    std::vector<double4> vconst(lp.n);
    for (int64_t v = 0; v < lp.n; ++v)
        vconst[v] = double4{lp.c[v], lp.lo[v], lp.hi[v], double(var_off[v + 1] - var_off[v])};
    h.s_vconst.upload(vconst, s, "upload streamed plan");
    h.s_part.alloc(size_t(2) * kSBlocks * 5, "streamed residual rows");
    h.s_u2.alloc(size_t(2) * nloc, "streamed x_s - lambda / rho, two buffers");
    h.s_lam2.alloc(size_t(nloc), "streamed lambda, second buffer");
    h.s_x2.alloc(size_t(2) * lp.n, "streamed x halves");
    h.s_ctrl.alloc(2, "streamed control");
    if (!h.s_hctrl)
        hip_check(hipHostMalloc(reinterpret_cast<void**>(&h.s_hctrl), 4 * sizeof(int64_t), hipHostMallocDefault),
                  "pinned control");
    for (hipEvent_t& e : h.s_evc)
        if (!e) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    h.s_nq = max_n <= 64 ? 1 : (max_n <= 256 ? 4 : 16);
    h.streamed = true;
    h.plan = Plan{};
    h.plan.rank_words = rank_words;
    h.plan.block_threads = 64 * kSWaves;
    drop_stream_graph(h);
}

void stream_solve(ldopf_problem& h) {
    // the graph holds the kernel arguments (options, buffers): capture anew
    // for every solve, which also follows option changes
    drop_stream_graph(h);
    const StreamArgs a = stream_args(h);
    hipStream_t s = h.stream;
    hipLaunchKernelGGL(stream_init_kernel, dim3(1), dim3(64), 0, s, a);
    hip_check(hipGetLastError(), "streamed sweep init");
    const unsigned cblocks = unsigned((a.nloc + 255) / 256);
    if (cblocks > 0) {
        // buffer 0 holds u of the starting point
        StreamArgs a0 = a;
        a0.u_wr = const_cast<double*>(a.u_rd);
        hipLaunchKernelGGL(stream_u_kernel, dim3(cblocks), dim3(256), 0, s, a0, h.xs.p, h.lam.p);
        hip_check(hipGetLastError(), "streamed sweep init");
    }
    const int rows = int(std::min<int64_t>(kSBlocks, std::max<int64_t>(1, (a.n_groups + kSWaves - 1) / kSWaves)));
    hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture");
    // node i of a graph computes sweep 32 g + i + 1 (every graph starts after
    // a multiple of kSGraph sweeps, an even number): it writes buffer
    // (i + 1) % 2 (x half, x_s, lambda, block sums) and reads the other
    for (int i = 0; i < kSGraph; ++i) {
        StreamArgs ai = a;
        const int wb = (i + 1) % 2;
        ai.x = a.x + int64_t(wb) * a.n;
        ai.u_rd = wb ? a.u_rd : a.u_wr;
        ai.lam_rd = wb ? a.lam_rd : a.lam_wr;
        ai.u_wr = wb ? a.u_wr : const_cast<double*>(a.u_rd);
        ai.lam_wr = wb ? a.lam_wr : const_cast<double*>(a.lam_rd);
        ai.part_rd = wb ? a.part_rd : a.part_wr;
        ai.part_wr = wb ? a.part_wr : const_cast<double*>(a.part_rd);
        void* args[] = {&ai, const_cast<int*>(&rows)};
        (void)hipLaunchKernel(sweep_kernel_for(h.s_nq), dim3(rows + 1), dim3(64 * kSWaves), args, 0, s);
    }
    hip_check(hipStreamEndCapture(s, &h.s_graph), "graph capture");
    hip_check(hipGraphInstantiate(&h.s_exec, h.s_graph, nullptr, nullptr, 0), "graph instantiate");
    // Each graph is followed by a read of the control words into pinned
    // memory and an event; the next graph is queued before the host waits
    // for the last one's words, so the host's round trip overlaps sweeps (a
    // graph queued after the stop returns at once).
    int64_t* hc = h.s_hctrl;
    auto queue = [&](int b) {
        hip_check(hipGraphLaunch(h.s_exec, s), "graph launch");
        hip_check(hipMemcpyAsync(hc + 2 * b, h.s_ctrl.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s),
                  "download control");
        hip_check(hipEventRecord(h.s_evc[b], s), "event");
    };
    int b = 0;
    int64_t before = 0, t = 0;
    queue(0);
    for (;;) {
        queue(b ^ 1);
        hip_check(hipEventSynchronize(h.s_evc[b]), "streamed sweep");
        t = hc[2 * b];
        if (hc[2 * b + 1]) break;
        // every sweep of a graph that did not stop advances the count
        if (t != before + kSGraph) fail(LDOPF_DEVICE_ERROR, "the streamed sweep count did not advance");
        before = t;
        b ^= 1;
    }
    // the state of the returned sweep (the sweep number when stopped) into
    // the handle's x, x_s (from u and lambda) and lambda, after the graph
    // queued last
    if (t >= 1)
        hip_check(hipMemcpyAsync(h.x.p, h.s_x2.p + (t % 2) * a.n, size_t(a.n) * 8, hipMemcpyDeviceToDevice, s),
                  "copy x");
    if (t >= 1 && cblocks > 0) {
        StreamArgs af = a;
        af.u_rd = t % 2 ? a.u_wr : a.u_rd;
        af.lam_rd = t % 2 ? a.lam_wr : a.lam_rd;
        hipLaunchKernelGGL(stream_xs_kernel, dim3(cblocks), dim3(256), 0, s, af, h.xs.p);
        hip_check(hipGetLastError(), "streamed x_s");
        if (t % 2 == 1)
            hip_check(hipMemcpyAsync(h.lam.p, h.s_lam2.p, size_t(a.nloc) * 8, hipMemcpyDeviceToDevice, s), "copy lambda");
    }
}

}  // namespace ldopf
