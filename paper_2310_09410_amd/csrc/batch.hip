// Batched scenarios: one network, B load scenarios, solved together.
//
// Scenario k multiplies the reference powers of every load l by f[k][l].
// That scales the right-hand side of the load's model rows and, for a
// voltage-dependent load (alpha or beta > 0), also the squared-voltage
// coefficient of those rows (Section II-A, VDLM-1 and VDLM-2). So:
//   * a subsystem with no voltage-dependent load has one operator for all
//     scenarios, kept in rank form (the K_s = min(r, n_s - r) orthonormal
//     rows W of the smaller of the row-space and complement bases, so that
//     -Abar_s v = v - W'(W v) or W'(W v)); its local update for B scenarios
//     is two small GEMMs, T = W V and W'T with V of size n_s x B, run on
//     MFMA (v_mfma_f32_16x16x4f32, 64-scenario tiles);
//   * a subsystem with one has a different operator per scenario; its update
//     runs in the same rank form per scenario (vector code,
//     scenario-contiguous data).
// bbar differs per scenario everywhere. Operators are precomputed in FP64 on
// the device for every (subsystem, scenario) pair and stored in FP32; the
// sweep (global update, local update, dual update) runs in FP32; residual
// sums, the termination test and the per-scenario masks in FP64. Each
// scenario stops at its own first sweep that passes the test (Section III-C)
// and keeps that state while the others continue. Two launches per sweep:
// the global update, whose first blocks also reduce the residual sums of the
// previous sweep and run its test, and the local update; the global update
// of sweep k writes x into the half k % 2 of a two-part buffer, so the x of
// a scenario's stopping sweep survives the next sweep's global update (the
// local update of that sweep skips the scenario, so its x_s and lambda stay
// too). C sweeps are captured in one HIP graph (C even, the half fixed per
// node); the host replays it until every scenario has stopped.
//
// State layout in HBM: row-major [copy or variable][scenario], scenarios
// padded to Bp (a multiple of 64), so a wave reads 64 consecutive scenarios.
// Each copy keeps lambda and u = x_s - lambda / rho instead of x_s: the
// global update needs only the sum of u over a variable's copies (one word
// per copy instead of two), and the local update forms the previous x_s =
// u + lambda / rho for the dual residual (the same FP32 arithmetic gives the
// same x; the reconstructed x_s differs from the computed one by the FP32
// rounding of the subtraction).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "device.h"
#include "gs_core.h"
#include "host_util.h"
#include "internal.h"

namespace ldopf {

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kTile = 64;  // scenarios per wave
constexpr int kZS = 80;    // LDS row stride (floats) of the local update
constexpr int kVPW = 8;    // variables per wave in the global update
constexpr int kRedBlocks = 16;  // reduction blocks (four waves each) per scenario tile
constexpr int kKB = 1;         // operator rows per load batch of the per-scenario class

struct PrecomputeBatchArgs {
    int64_t S, nloc, words;
    int32_t k0, C, n_load;
    const int32_t* ns;
    const int32_t* ms;
    const int64_t* a_off;
    const int64_t* row_off;
    const int64_t* loc_off;
    const int64_t* basis_off;
    const double* A;
    const double* b;
    const int32_t* row_load;
    const int32_t* row_wcol;
    const double* scale;  // [B][n_load]
    double* tmp_basis;    // [C][words]
    double* tmp_bbar;     // [C][nloc]
    int32_t* tmp_rank;    // [C][S]
    int32_t* tmp_bad;     // [C][S]
    double tol_dep, tol_rhs;
};

struct PackArgs {
    int64_t S, nloc, words;
    int32_t k0, C, Bp;
    const int32_t* ns;
    const int64_t* loc_off;
    const int64_t* basis_off;
    const int32_t* rank;      // rank at unit scale
    const int32_t* cls;       // 0 MFMA, 1 vector
    const int32_t* vK;
    const int32_t* vbrow;
    const int64_t* wofs;      // first W row (units of Bp) of a vector-class subsystem
    const double* tmp_basis;
    const double* tmp_bbar;
    const int32_t* tmp_rank;
    const int32_t* tmp_bad;
    float* BB;
    float* W;
    int32_t* flag;            // bit 1: rank changed with the scale, bit 2: inconsistent rows
};

// Read-only tables of a kernel read through the constant address space, so
// that uniform reads become scalar loads.
template <typename T>
using CPtr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ inline CPtr<T> as_const(const T* p) {
    return (CPtr<T>)(p);
}

// One subsystem of the local update: n_s, class (0 shared operator on MFMA,
// 1 per-scenario rank form), K_s and mode of the rank form, first copy, and
// the offset of its shared Abar_s (class 0, floats) or of its first W row
// (class 1, units of the padded scenario count).
struct LocalMeta {
    int32_t n, cls, K, mode;
    int64_t row0, off;
};
static_assert(sizeof(LocalMeta) == 32, "LocalMeta layout");

__device__ inline LocalMeta load_meta(CPtr<int32_t> t, int q) {
    const CPtr<int32_t> e = t + 8 * q;
    LocalMeta m;
    m.n = e[0];
    m.cls = e[1];
    m.K = e[2];
    m.mode = e[3];
    m.row0 = int64_t(uint32_t(e[4])) | (int64_t(e[5]) << 32);
    m.off = int64_t(uint32_t(e[6])) | (int64_t(e[7]) << 32);
    return m;
}

struct BatchArgs {
    int32_t B, Bp;
    int64_t n, nloc;
    const int32_t* ns;
    const int64_t* loc_off;
    const int32_t* gidx;
    const int32_t* var_off;
    const int32_t* var_copy;
    const float* crho;
    const float* lo;
    const float* hi;
    const float* invN;
    float* X;  // the half of the two-part x buffer this sweep writes (global) and reads (local)
    float* U;  // per copy and scenario: u = x_s - lambda / rho (so x_s = u + lambda / rho)
    float* LAM;
    const float* BB;
    const int4* ell;      // [n] first four copies of each variable, -1 padded
    // local update: chunks of subsystems, both classes
    int32_t n_chunks;
    const int32_t* chunk_off;
    const LocalMeta* meta;  // per subsystem, in chunk order
    int32_t nmax, kmax;     // largest n_s, largest K_s of the per-scenario class
    const float* ash;       // shared FP32 Abar_s
    const float* W;         // per-scenario rank-form rows
    // residuals and control
    double* part;      // [part_rows][5][Bp]
    int32_t part_rows;
    double* part2;     // [tiles][kRedBlocks][5][64] slice sums of the reduction
    int32_t* tick;     // [tiles] reduction blocks finished, per tile
    int32_t* active;   // [Bp]
    int32_t* conv;     // [Bp]
    int64_t* iters;    // [Bp]
    double* res;       // [Bp][4]
    int32_t* sflags;   // [Bp]
    int64_t* ctrl;     // [0] the sweep being computed (tested by the next global update), [1] all done,
                       // [2] active count, [3] arrivals
    int64_t max_iter;
    int32_t check;
    double rho, eps_rel, eps_abs;
};

__global__ __launch_bounds__(256) void precompute_batch_kernel(PrecomputeBatchArgs a) {
    __shared__ double sbeta[4][256];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t v = int64_t(blockIdx.x) * 4 + wv;
    if (v >= a.S * a.C) return;
    const int64_t s = v % a.S;
    const int64_t kc = v / a.S;
    const int64_t k = a.k0 + kc;
    const double* fs = a.n_load > 0 ? a.scale + k * a.n_load : nullptr;
    int bad = 0;
    const int r = gs_project<4>(lane, a.ns[s], a.ms[s], a.A + a.a_off[s], a.b + a.row_off[s], a.row_load + a.row_off[s],
                             a.row_wcol + a.row_off[s], fs, a.tol_dep, a.tol_rhs,
                             a.tmp_basis + kc * a.words + a.basis_off[s], sbeta[wv],
                             a.tmp_bbar + kc * a.nloc + a.loc_off[s], nullptr, &bad);
    if (lane == 0) {
        a.tmp_rank[kc * a.S + s] = r;
        a.tmp_bad[kc * a.S + s] = bad;
    }
}

__global__ __launch_bounds__(256) void batch_pack_kernel(PackArgs a) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t v = int64_t(blockIdx.x) * 4 + wv;
    if (v >= a.S * a.C) return;
    const int64_t s = v % a.S;
    const int64_t kc = v / a.S;
    const int64_t k = a.k0 + kc;
    const int n = a.ns[s];
    if (lane == 0) {
        if (a.tmp_rank[kc * a.S + s] != a.rank[s]) atomicOr(a.flag, 1);
        if (a.tmp_bad[kc * a.S + s]) atomicOr(a.flag, 2);
    }
    const double* bb = a.tmp_bbar + kc * a.nloc + a.loc_off[s];
    for (int j = lane; j < n; j += 64) a.BB[(a.loc_off[s] + j) * a.Bp + k] = float(bb[j]);
    if (a.cls[s] == 1) {
        const int K = a.vK[s], brow = a.vbrow[s];
        const double* U = a.tmp_basis + kc * a.words + a.basis_off[s];
        for (int idx = lane; idx < K * n; idx += 64) {
            const int kk = idx / n, jj = idx - kk * n;
            a.W[(a.wofs[s] + idx) * a.Bp + k] = float(U[int64_t(brow + kk) * n + jj]);
        }
    }
}

// Residual sums per scenario over the local blocks' partial rows of the
// previous sweep, and its termination test, in the first blocks of the next
// global update (beside the blocks of the update itself). Two levels:
// kRedBlocks blocks per scenario tile each add a contiguous slice of the rows
// (wave w adds rows w, w + 4, ...; then the four waves in order) and store
// the slice sums; the last block of the tile to finish (a ticket per tile)
// adds the slices in order and runs the test and the masks; the last tile to
// finish either stops the batch or numbers the sweep the update computes.
// The order of every sum is fixed. The update blocks of the same launch may
// or may not see a scenario stop: either way they write the other half of x,
// and the local update after them sees the masks.
// Words read by other blocks of the same launch (the slice sums) go through
// the device's coherence point (agent-scope relaxed atomics); a block makes
// them visible before it takes its ticket by waiting for its own stores to
// complete (s_waitcnt 0) instead of a device-scope release fence, which would
// write back the whole L2 of its XCD.
__device__ inline void st_dev(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_dev(const double* p) {
    return __longlong_as_double((long long)__hip_atomic_load(
        reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ inline void batch_test(const BatchArgs& a, int rblock) {
    __shared__ double red[4][5][kTile];
    __shared__ int last;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles = a.Bp / kTile;
    const int tile = rblock / kRedBlocks, rb = rblock % kRedBlocks;
    const int sc = tile * kTile + lane;
    // the sweep the previous local update computed (0 before the first one);
    // used before this block's ticket, so read before the last block of the
    // launch changes it
    const int64_t t = a.ctrl[0];
    // a tile whose scenarios have all stopped reads nothing, but still
    // arrives at the counts below
    const bool any = __syncthreads_or(t >= 1 && a.active[sc] != 0);
    const int per = (a.part_rows + kRedBlocks - 1) / kRedBlocks;
    const int r0 = min(a.part_rows, rb * per), r1 = any ? min(a.part_rows, r0 + per) : r0;
    double acc[5] = {0, 0, 0, 0, 0};
    int r = r0 + wv;
    for (; r + 4 < r1; r += 8) {
        double u[5], w[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            u[q] = a.part[(int64_t(r) * 5 + q) * a.Bp + sc];
            w[q] = a.part[(int64_t(r + 4) * 5 + q) * a.Bp + sc];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] += u[q] + w[q];
    }
    if (r < r1)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] += a.part[(int64_t(r) * 5 + q) * a.Bp + sc];
#pragma unroll
    for (int q = 0; q < 5; ++q) red[wv][q][lane] = acc[q];
    __syncthreads();
    double* slice = a.part2 + int64_t(tile) * kRedBlocks * 5 * kTile;
    if (wv == 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q)
            st_dev(slice + (rb * 5 + q) * kTile + lane,
                   ((red[0][q][lane] + red[1][q][lane]) + red[2][q][lane]) + red[3][q][lane]);
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(&a.tick[tile], 1) == kRedBlocks - 1;
    __syncthreads();
    if (!last) return;
    if (wv == 0) {
        int still = sc < a.B && a.active[sc] != 0;
        if (t >= 1 && still) {
            double d[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                double u = 0.0;
                for (int b2 = 0; b2 < kRedBlocks; ++b2) u += ld_dev(slice + (b2 * 5 + q) * kTile + lane);
                d[q] = u;
            }
            const double sq = sqrt(double(a.nloc));
            const double pres = sqrt(d[0]), dres = a.rho * sqrt(d[1]);
            const double eps_p = sq * a.eps_abs + a.eps_rel * fmax(sqrt(d[2]), sqrt(d[3]));
            const double eps_d = sq * a.eps_abs + a.eps_rel * sqrt(d[4]);
            a.iters[sc] = t;
            a.res[sc * 4 + 0] = pres;
            a.res[sc * 4 + 1] = dres;
            a.res[sc * 4 + 2] = eps_p;
            a.res[sc * 4 + 3] = eps_d;
            const bool conv = pres <= eps_p && dres <= eps_d;
            a.conv[sc] = conv;
            const bool bad = !isfinite(d[0] + d[1] + d[2] + d[3] + d[4]);
            if (bad) a.sflags[sc] |= 2;
            still = !(bad || (a.check && conv));
            if (!still) a.active[sc] = 0;
        }
        const unsigned long long ball = __ballot(still);
        if (lane == 0) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.ctrl[2]), (unsigned long long)__popcll(ball));
            a.tick[tile] = 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned long long prev = atomicAdd(reinterpret_cast<unsigned long long*>(&a.ctrl[3]), 1ull);
        if (prev == unsigned(tiles) - 1) {
            const long long left = atomicAdd(reinterpret_cast<unsigned long long*>(&a.ctrl[2]), 0ull);
            a.ctrl[2] = 0;
            a.ctrl[3] = 0;
            if (t >= 1 && (left == 0 || t >= a.max_iter))
                a.ctrl[1] = 1;
            else
                a.ctrl[0] = t + 1;
        }
    }
}

// Global update (closed_1): a wave takes kVPW consecutive variables for one
// 64-scenario tile; the four waves of a block take the same variables for
// four tiles. The first four copies of each variable come from a padded
// table (one 16-byte read per variable) so that all their loads are in flight
// together; further copies, if any, from the CSR lists. Copies are added in
// CSR order. The first kRedBlocks blocks per tile run the test of the
// previous sweep instead.
__global__ __launch_bounds__(256) void batch_global_kernel(BatchArgs a) {
    if (a.ctrl[1]) return;
    const int n_red = (a.Bp / kTile) * kRedBlocks;
    if (int(blockIdx.x) < n_red) {
        batch_test(a, int(blockIdx.x));
        return;
    }
    const int lane = threadIdx.x & 63;
    const int64_t nvb = (a.n + kVPW - 1) / kVPW, b = int64_t(blockIdx.x) - n_red;
    const int64_t v0 = (b % nvb) * kVPW;
    const int tile = int(b / nvb) * 4 + (threadIdx.x >> 6);
    if (tile * kTile >= a.Bp) return;
    const int sc = tile * kTile + lane;
    if (v0 >= a.n || !a.active[sc]) return;
    const int64_t Bp = a.Bp;
    // the copies' x_s - lambda / rho, as the local update left them
    float uc[kVPW][4];
#pragma unroll
    for (int u = 0; u < kVPW; ++u) {
        const int64_t v = v0 + u;
        const int4 e = v < a.n ? a.ell[v] : int4{-1, -1, -1, -1};
        const int ec[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) uc[u][i] = ec[i] >= 0 ? a.U[int64_t(ec[i]) * Bp + sc] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kVPW; ++u) {
        const int64_t v = v0 + u;
        if (v >= a.n) break;
        const int q0 = a.var_off[v], q1 = a.var_off[v + 1];
        float s = uc[u][0];
#pragma unroll
        for (int i = 1; i < 4; ++i)
            if (q0 + i < q1) s += uc[u][i];
        for (int q = q0 + 4; q < q1; ++q) s += a.U[int64_t(a.var_copy[q]) * Bp + sc];
        float x = (s - a.crho[v]) * a.invN[v];
        x = x < a.lo[v] ? a.lo[v] : x;
        x = x > a.hi[v] ? a.hi[v] : x;
        a.X[v * Bp + sc] = x;
    }
}

// Local + dual update of both classes, four waves per block on one
// 64-scenario tile (lane = scenario). Rows j of a subsystem belong to wave
// j % 4; a wave keeps its rows' z, lambda and old u in registers (at most
// RPW rows, so n_s <= 4 RPW) and stages v = z + lambda / rho and bbar, then
// the projection y, in LDS ([row][kZS], kZS = 80 floats: rows four apart fall on
// disjoint halves of the 32 banks, so the MFMA operand reads do not
// conflict).
//   shared-operator class: T = W V, then Y = Bbar + V - W'T (mode 1) or
//     Bbar + W'T (mode 0), both on MFMA; wave w takes the 16-row tiles w,
//     w + 4, ... of the product against the four 16-scenario tiles;
//     v_mfma_f32_16x16x4f32 operand layout: lane l holds A[l % 16][l / 16],
//     B[l / 16][l % 16] and D[4 (l / 16) + i][l % 16], i < 4;
//   per-scenario class: t = W v (wave w takes basis rows w, w + 4, ...), then
//     y = bbar + v - W't (mode 1) or bbar + W't (mode 0) per row.
// Then lambda += rho (z - y), u = y - lambda / rho, and the FP64 residual
// sums per scenario.
// Four blocks per CU (four waves per SIMD, at most 128 VGPRs) for the common
// subsystem width: the phases of a subsystem (row loads, MFMA or operator
// streams, barriers) then overlap across blocks. The wider variants keep
// their registers instead (a cap would make them spill).
template <int RPW>
__global__ __launch_bounds__(256, RPW <= 10 ? 4 : 1) void batch_local_kernel(BatchArgs a) {
    if (a.ctrl[1]) return;
    extern __shared__ __align__(16) float sm[];
    float* Vs = sm;                         // [nmax][kZS]
    float* Ys = Vs + a.nmax * kZS;          // [nmax][kZS]
    float* Ts = Ys + a.nmax * kZS;          // [kmax][kZS]
    float* As = Ts + a.kmax * kZS;          // [kmax * nmax] shared rank-form rows
    const int tid = threadIdx.x, lane_id = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int Bp = a.Bp;
    // the scenario tiles of one chunk-block are adjacent block ids, so the
    // quarters of each row are read at about the same time
    const int tiles = a.Bp / kTile;
    const int tile = int(blockIdx.x) % tiles, bx = int(blockIdx.x) / tiles, nbx = int(gridDim.x) / tiles;
    const int sc_id = tile * kTile + lane_id;
    const bool on = a.active[sc_id] != 0;
    // a tile whose scenarios have all stopped is skipped (its partial rows
    // are not read: the test runs only for active scenarios)
    if (__syncthreads_or(on) == 0) return;
    const float rho = float(a.rho), irho = float(1.0 / a.rho);
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, p4 = 0.0;
    // read-only tables through the constant address space (scalar loads)
    const CPtr<int32_t> chunk_off = as_const(a.chunk_off);
    const CPtr<int32_t> meta = as_const(reinterpret_cast<const int32_t*>(a.meta));
    const CPtr<int32_t> gidx = as_const(a.gidx);
    bool prev_shared = false;  // the last subsystem was of the shared-operator class
    for (int c = bx; c < a.n_chunks; c += nbx) {
        const int q1 = chunk_off[c + 1];
        int q = chunk_off[c];
        LocalMeta m = load_meta(meta, q);
        for (; q < q1; ++q) {
            // opaque copies of the lane's indices, so that per-lane addresses
            // are formed again in each subsystem instead of being held across
            // the loop (they would not fit the register budget)
            int lane_o = lane_id, sc_o = sc_id;
            asm volatile("" : "+v"(lane_o), "+v"(sc_o));
            const int lane = lane_o, sc = sc_o;
            // the next subsystem's metadata is loaded one subsystem ahead
            const LocalMeta mn = load_meta(meta, q + 1 < q1 ? q + 1 : q);
            const int n = m.n;
            const int64_t row0 = m.row0;
            const float* LAMb = a.LAM + row0 * Bp;
            const float* Ub = a.U + row0 * Bp;
            const float* BBb = a.BB + row0 * Bp;
            // row indices first, then every row load of the wave before any
            // use; rows past n_s repeat the last row (loaded, never used) so
            // that no branch separates the loads
            int gi[RPW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) gi[r] = gidx[row0 + min(wv + 4 * r, n - 1)];
            float z[RPW], l0[RPW], xo[RPW], bb[RPW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int o = min(wv + 4 * r, n - 1) * Bp + sc;
                z[r] = a.X[gi[r] * Bp + sc];
                l0[r] = LAMb[o];
                xo[r] = Ub[o];  // u of the previous sweep; x_s = u + lambda / rho
                bb[r] = BBb[o];
            }
            float y[RPW];
            if (m.cls == 0) {
                const float* Ab = a.ash + m.off;
                for (int i = tid; i < m.K * n; i += 256) As[i] = Ab[i];
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const int j = wv + 4 * r;
                    if (j < n) {
                        Vs[j * kZS + lane] = z[r] + l0[r] * irho;
                        Ys[j * kZS + lane] = bb[r];
                    }
                }
                __syncthreads();
                // T = W V: (16-row tile of W, 16-scenario tile) products spread
                // over the four waves
                const int K = m.K, mode = m.mode;
                for (int pq = wv; pq < ((K + 15) >> 4) * 4; pq += 4) {
                    const int mt = pq >> 2, nt = pq & 3;
                    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
                    const int ar = mt * 16 + (lane & 15);
                    for (int kk = 0; kk * 4 < n; ++kk) {
                        const int kc = kk * 4 + (lane >> 4);
                        const bool in = kc < n;
                        const float av = (ar < K && in) ? As[ar * n + kc] : 0.f;
                        const float bv = in ? Vs[kc * kZS + nt * 16 + (lane & 15)] : 0.f;
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = mt * 16 + 4 * (lane >> 4) + i;
                        if (row < K) Ts[row * kZS + nt * 16 + (lane & 15)] = acc[i];
                    }
                }
                __syncthreads();
                // U = W' T, then y = bbar + v - U (mode 1) or bbar + U (mode 0),
                // the tile products spread over the waves the same way
                for (int pq = wv; pq < ((n + 15) >> 4) * 4; pq += 4) {
                    const int mt = pq >> 2, nt = pq & 3;
                    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
                    const int ar = mt * 16 + (lane & 15);
                    for (int kk = 0; kk * 4 < K; ++kk) {
                        const int kc = kk * 4 + (lane >> 4);
                        const bool in = kc < K;
                        const float av = (ar < n && in) ? As[kc * n + ar] : 0.f;
                        const float bv = in ? Ts[kc * kZS + nt * 16 + (lane & 15)] : 0.f;
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = mt * 16 + 4 * (lane >> 4) + i;
                        if (row < n) {
                            const int e = row * kZS + nt * 16 + (lane & 15);
                            Ys[e] = mode ? Ys[e] + (Vs[e] - acc[i]) : Ys[e] + acc[i];
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RPW; ++r) y[r] = Ys[min(wv + 4 * r, n - 1) * kZS + lane];
                prev_shared = true;
            } else {
                // Per-scenario operator, on the wave's own rows j = wv + 4 r with
                // v_j in registers: each wave adds its rows' terms of t = W v
                // for every k (partial sums in LDS, over the rows of v and y,
                // which this class does not use), then, after one barrier, t_k
                // = the four partials in wave order and y_j = bbar_j + v_j -
                // sum_k W_kj t_k (mode 1) or bbar_j + sum_k W_kj t_k (mode 0).
                // W is read in batches of kKB operator rows x RPW rows, all
                // loads of a batch issued together and the next batch issued
                // before the current one is used.
                const int K = m.K, mode = m.mode;
                float* Tp = Vs;  // [4][K][64]
                // the shared class before reads its y rows after its last
                // barrier: wait for every wave before the partials overwrite them
                if (prev_shared) __syncthreads();
                prev_shared = false;
                // v_j = z_j + lambda_j / rho, recomputed where used; zero past n_s
                auto vj = [&](int r) -> float { return (wv + 4 * r < n) ? z[r] + l0[r] * irho : 0.f; };
                if (K == 0) {
#pragma unroll
                    for (int r = 0; r < RPW; ++r) y[r] = mode ? bb[r] + vj(r) : bb[r];
                } else {
                    // W row (k, j) at (k n_s + j) Bp + sc. A batch takes rows
                    // k0 .. k0 + kKB - 1 of W for the wave's RPW rows j; rows past
                    // the subsystem (k >= K, or j >= n_s) read the last row that
                    // exists again (a cache hit), so every batch issues the same
                    // loads and stays inside the subsystem's operator
                    const char* Wc = reinterpret_cast<const char*>(a.W + m.off * Bp);
                    const uint32_t Bp4 = uint32_t(Bp) * 4u;
                    const uint32_t jo = uint32_t(sc) * 4u;
                    const int nr = max(1, (n - wv + 3) / 4);  // the wave's rows
                    auto issue = [&](float (&w)[kKB][RPW], int k0) {
#pragma unroll
                        for (int kb = 0; kb < kKB; ++kb)
#pragma unroll
                            for (int r = 0; r < RPW; ++r) {
                                // uniform base (scalar registers) + the lane's 32-bit offset
                                const int k = min(k0 + kb, K - 1), j = min(wv + 4 * min(r, nr - 1), n - 1);
                                const char* base = Wc + uint32_t(k * n + j) * Bp4;
                                w[kb][r] = *reinterpret_cast<const float*>(base + jo);
                            }
                    };
                    auto t_use = [&](const float (&w)[kKB][RPW], int k0) {
#pragma unroll
                        for (int kb = 0; kb < kKB; ++kb) {
                            float t = 0.f;
#pragma unroll
                            for (int r = 0; r < RPW; ++r) t += w[kb][r] * vj(r);
                            if (k0 + kb < K) Tp[(wv * K + k0 + kb) * 64 + lane] = t;
                        }
                    };
                    float acc[RPW];
#pragma unroll
                    for (int r = 0; r < RPW; ++r) acc[r] = 0.f;
                    auto y_use = [&](const float (&w)[kKB][RPW], int k0) {
#pragma unroll
                        for (int kb = 0; kb < kKB; ++kb) {
                            const int k = min(k0 + kb, K - 1);
                            const float tk = ((Tp[(0 * K + k) * 64 + lane] + Tp[(1 * K + k) * 64 + lane]) +
                                              Tp[(2 * K + k) * 64 + lane]) +
                                             Tp[(3 * K + k) * 64 + lane];
                            const float g = k0 + kb < K ? tk : 0.f;
#pragma unroll
                            for (int r = 0; r < RPW; ++r) acc[r] += w[kb][r] * g;
                        }
                    };
                    // loads are issued on every path (never behind a branch),
                    // so the wait before each use counts only older batches
                    float wa[kKB][RPW], wb[kKB][RPW];
                    issue(wa, 0);
                    for (int k0 = 0;; k0 += 2 * kKB) {
                        issue(wb, k0 + kKB);
                        t_use(wa, k0);
                        if (k0 + kKB >= K) break;
                        issue(wa, k0 + 2 * kKB);
                        t_use(wb, k0 + kKB);
                        if (k0 + 2 * kKB >= K) break;
                    }
                    if (K <= kKB) {
                        // the one batch is still held in wa
                        __syncthreads();
                        y_use(wa, 0);
                    } else {
                        issue(wa, 0);
                        __syncthreads();
                        for (int k0 = 0;; k0 += 2 * kKB) {
                            issue(wb, k0 + kKB);
                            y_use(wa, k0);
                            if (k0 + kKB >= K) break;
                            issue(wa, k0 + 2 * kKB);
                            y_use(wb, k0 + kKB);
                            if (k0 + 2 * kKB >= K) break;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < RPW; ++r) y[r] = mode ? bb[r] + (vj(r) - acc[r]) : bb[r] + acc[r];
                    // every wave has read the partials before the next subsystem writes them
                    __syncthreads();
                }
            }
            // dual update and residual sums on the wave's own rows
            float* Uw = a.U + row0 * Bp;
            float* LAMw = a.LAM + row0 * Bp;
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int j = wv + 4 * r;
                if (j < n && on) {
                    const int o = j * Bp + sc;
                    const float yj = y[r];
                    const float l1 = l0[r] + rho * (z[r] - yj);
                    Uw[o] = yj - l1 * irho;
                    LAMw[o] = l1;
                    const float xprev = xo[r] + l0[r] * irho;
                    const double dz = double(z[r]) - double(yj), dx = double(yj) - double(xprev);
                    p0 += dz * dz;
                    p1 += dx * dx;
                    p2 += double(z[r]) * double(z[r]);
                    p3 += double(yj) * double(yj);
                    p4 += double(l1) * double(l1);
                }
            }
            m = mn;
        }
    }
    // the four waves' sums of each scenario, in wave order
    __syncthreads();
    double* red = reinterpret_cast<double*>(sm);  // [4][5][64]
    red[(wv * 5 + 0) * 64 + lane_id] = p0;
    red[(wv * 5 + 1) * 64 + lane_id] = p1;
    red[(wv * 5 + 2) * 64 + lane_id] = p2;
    red[(wv * 5 + 3) * 64 + lane_id] = p3;
    red[(wv * 5 + 4) * 64 + lane_id] = p4;
    __syncthreads();
    double* out = a.part + int64_t(bx) * 5 * Bp;
    for (int e = tid; e < 5 * 64; e += 256) {
        const int qq = e >> 6, l = e & 63;
        out[qq * Bp + tile * kTile + l] = ((red[(0 * 5 + qq) * 64 + l] + red[(1 * 5 + qq) * 64 + l]) +
                                                 red[(2 * 5 + qq) * 64 + l]) +
                                                red[(3 * 5 + qq) * 64 + l];
    }
}

__global__ void batch_init_kernel(BatchArgs a, const double* x_init) {
    // initial point of Section V-A for every scenario; plain stores
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = a.nloc * a.Bp;
    if (i < total) {
        const int64_t c = i / a.Bp;
        a.U[i] = float(x_init[a.gidx[c]]);  // lambda = 0: u = x_s
        a.LAM[i] = 0.f;
    }
    if (i < 2 * a.n * a.Bp) a.X[i] = 0.f;  // both halves
    if (i < a.Bp) {
        const int sc = int(i);
        a.active[sc] = sc < a.B ? 1 : 0;
        a.conv[sc] = 0;
        a.iters[sc] = 0;
        a.sflags[sc] = 0;
        for (int q = 0; q < 4; ++q) a.res[sc * 4 + q] = 0.0;
    }
    if (i < 4) a.ctrl[i] = 0;
    if (i < a.Bp / kTile) a.tick[i] = 0;
}

}  // namespace

}  // namespace ldopf

using namespace ldopf;

struct ldopf_batch {
    ConsensusLP lp;
    ldopf_options opts{};
    int32_t B = 0, Bp = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t* hctrl = nullptr;                 // pinned: the control words after two graphs
    hipEvent_t evc[2] = {nullptr, nullptr};  // recorded after each of those reads
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t graph_sweeps = 16;
    int32_t grid = 0;         // local-update blocks per scenario tile
    int32_t nmax = 1, kmax = 1, rpw = 10;
    int64_t w_words = 0;  // FP32 words of the per-scenario operators (without the padding)
    double precompute_ms = 0.0;
    int64_t n_mf = 0, n_vec = 0;
    std::vector<int32_t> chunk_off_h;
    int32_t rows_per_chunk = 0;

    DevBuf<int32_t> ns, gidx, var_off, var_copy, chunk_off, cls, vK;
    DevBuf<LocalMeta> meta;
    std::vector<LocalMeta> meta_h;  // per subsystem, in subsystem order
    DevBuf<int4> ell;
    DevBuf<int64_t> loc_off, wofs, iters, ctrl;
    DevBuf<float> crho, lo, hi, invN, X, U, LAM, BB, ash, W;
    DevBuf<double> x_init, part, part2, res;
    DevBuf<int32_t> active, conv, sflags, tick;

    ~ldopf_batch() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        for (hipEvent_t e : evc)
            if (e) (void)hipEventDestroy(e);
        if (hctrl) (void)hipHostFree(hctrl);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

BatchArgs batch_args(ldopf_batch& h) {
    BatchArgs a{};
    a.B = h.B;
    a.Bp = h.Bp;
    a.n = h.lp.n;
    a.nloc = int64_t(h.lp.gidx.size());
    a.ns = h.ns.p;
    a.loc_off = h.loc_off.p;
    a.gidx = h.gidx.p;
    a.var_off = h.var_off.p;
    a.var_copy = h.var_copy.p;
    a.crho = h.crho.p;
    a.lo = h.lo.p;
    a.hi = h.hi.p;
    a.invN = h.invN.p;
    a.X = h.X.p;
    a.U = h.U.p;
    a.LAM = h.LAM.p;
    a.BB = h.BB.p;
    a.ell = h.ell.p;
    a.n_chunks = int32_t(h.chunk_off_h.size()) - 1;
    a.chunk_off = h.chunk_off.p;
    a.meta = h.meta.p;
    a.nmax = h.nmax;
    a.kmax = h.kmax;
    a.ash = h.ash.p;
    a.W = h.W.p;
    a.part = h.part.p;
    a.part_rows = h.grid;
    a.part2 = h.part2.p;
    a.tick = h.tick.p;
    a.active = h.active.p;
    a.conv = h.conv.p;
    a.iters = h.iters.p;
    a.res = h.res.p;
    a.sflags = h.sflags.p;
    a.ctrl = h.ctrl.p;
    a.max_iter = h.opts.max_iter;
    a.check = h.opts.check_termination;
    a.rho = h.opts.rho;
    a.eps_rel = h.opts.eps_rel;
    a.eps_abs = h.opts.eps_abs;
    return a;
}

size_t local_lds(const ldopf_batch& h) {
    return std::max<size_t>(size_t((2 * h.nmax + h.kmax) * kZS + h.nmax * h.kmax) * 4, size_t(4 * 5 * 64) * 8);
}

const void* local_kernel(int rpw) {
    switch (rpw) {
        case 10: return reinterpret_cast<const void*>(&batch_local_kernel<10>);
        case 16: return reinterpret_cast<const void*>(&batch_local_kernel<16>);
        default: return reinterpret_cast<const void*>(&batch_local_kernel<32>);
    }
}

void enqueue_sweep(ldopf_batch& h, const BatchArgs& a) {
    const int tiles = h.Bp / kTile;
    // the test blocks first, then the update blocks: a block's four waves
    // take the same variables for four scenario tiles, so that the four
    // quarters of each copy row are read together
    const int64_t update_blocks = (a.n + kVPW - 1) / kVPW * ((tiles + 3) / 4);
    hipLaunchKernelGGL(batch_global_kernel, dim3(unsigned(tiles * kRedBlocks + update_blocks)), dim3(256), 0, h.stream, a);
    BatchArgs copy = a;
    void* args[] = {&copy};
    (void)hipLaunchKernel(local_kernel(h.rpw), dim3(h.grid * tiles), dim3(256), args, local_lds(h), h.stream);
}

// Chunks of the subsystem order: consecutive subsystems up to rows_per_chunk copies.
std::vector<int32_t> make_chunks(const ConsensusLP& lp, int32_t rows_per_chunk) {
    std::vector<int32_t> off{0};
    int64_t rows = 0;
    for (int64_t q = 0; q < lp.S; ++q) {
        rows += lp.ns[q];
        if (rows >= rows_per_chunk) {
            off.push_back(int32_t(q + 1));
            rows = 0;
        }
    }
    if (off.back() != int32_t(lp.S)) off.push_back(int32_t(lp.S));
    return off;
}

// The captured graph holds the kernel arguments (options, chunking): drop it
// whenever they change.
void drop_graph(ldopf_batch& h) {
    if (h.exec) {
        (void)hipGraphExecDestroy(h.exec);
        h.exec = nullptr;
    }
    if (h.graph) {
        (void)hipGraphDestroy(h.graph);
        h.graph = nullptr;
    }
}

void set_chunks(ldopf_batch& h, int32_t rows_per_chunk, int32_t blocks_per_tile) {
    h.rows_per_chunk = rows_per_chunk;
    h.chunk_off_h = make_chunks(h.lp, rows_per_chunk);
    const int32_t nch = int32_t(h.chunk_off_h.size()) - 1;
    h.grid = std::max(1, std::min(nch, blocks_per_tile));
    h.chunk_off.upload(h.chunk_off_h, h.stream, "upload chunks");
    // within a chunk the shared-operator subsystems come first: a block
    // then switches class once per chunk (a switch to the per-scenario
    // class costs a barrier)
    std::vector<LocalMeta> ordered;
    ordered.reserve(h.meta_h.size());
    for (int32_t c = 0; c + 1 < int32_t(h.chunk_off_h.size()); ++c)
        for (int32_t cls : {0, 1})
            for (int32_t q = h.chunk_off_h[c]; q < h.chunk_off_h[c + 1]; ++q)
                if (h.meta_h[q].cls == cls) ordered.push_back(h.meta_h[q]);
    h.meta.upload(ordered, h.stream, "upload subsystems");
    h.part.alloc(size_t(h.grid) * 5 * h.Bp, "residual partials");
    drop_graph(h);
}

void build_graph(ldopf_batch& h) {
    if (h.exec) return;
    const BatchArgs a = batch_args(h);
    hip_check(hipStreamBeginCapture(h.stream, hipStreamCaptureModeThreadLocal), "graph capture");
    // node i computes sweep C g + i + 1 of the g-th replay: x half (i + 1) % 2
    for (int i = 0; i < h.graph_sweeps; ++i) {
        BatchArgs ai = a;
        ai.X = a.X + int64_t((i + 1) & 1) * a.n * a.Bp;
        enqueue_sweep(h, ai);
    }
    hip_check(hipStreamEndCapture(h.stream, &h.graph), "graph capture");
    hip_check(hipGraphInstantiate(&h.exec, h.graph, nullptr, nullptr, 0), "graph instantiate");
}

void batch_reset(ldopf_batch& h) {
    const BatchArgs a = batch_args(h);
    const int64_t total = std::max<int64_t>(int64_t(h.lp.gidx.size()), 2 * h.lp.n) * h.Bp;
    hipLaunchKernelGGL(batch_init_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, h.stream, a, h.x_init.p);
    hip_check(hipGetLastError(), "batch init");
    hip_check(hipStreamSynchronize(h.stream), "batch init");
}

// Runs the graph until every scenario stopped (or max_iter); returns sweeps.
int64_t run_to_done(ldopf_batch& h, double* ms_out) {
    if (ms_out) *ms_out = 0.0;
    if (h.opts.max_iter == 0) return 0;
    build_graph(h);
    int64_t ctrl[2] = {0, 0};
    hip_check(hipMemcpyAsync(ctrl, h.ctrl.p, sizeof(ctrl), hipMemcpyDeviceToHost, h.stream), "download control");
    hip_check(hipStreamSynchronize(h.stream), "download control");
    hip_check(hipEventRecord(h.ev0, h.stream), "event");
    // Each graph is followed by a read of the control words into pinned
    // memory and an event; the next graph is queued before the host waits
    // for the last one's words, so the host's round trip overlaps sweeps (a
    // graph queued after the stop returns at once).
    int64_t* hc = h.hctrl;
    auto queue = [&](int b) {
        hip_check(hipGraphLaunch(h.exec, h.stream), "graph launch");
        hip_check(hipMemcpyAsync(hc + 2 * b, h.ctrl.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, h.stream),
                  "download control");
        hip_check(hipEventRecord(h.evc[b], h.stream), "event");
    };
    int b = 0;
    int64_t before = ctrl[0];
    queue(0);
    for (;;) {
        queue(b ^ 1);
        hip_check(hipEventSynchronize(h.evc[b]), "batch sweep");
        ctrl[0] = hc[2 * b];
        ctrl[1] = hc[2 * b + 1];
        if (ctrl[1]) break;
        // every sweep of a graph that did not finish the batch advances the count
        if (ctrl[0] != before + h.graph_sweeps) fail(LDOPF_DEVICE_ERROR, "the batched sweep count did not advance");
        before = ctrl[0];
        b ^= 1;
    }
    hip_check(hipEventRecord(h.ev1, h.stream), "event");
    hip_check(hipEventSynchronize(h.ev1), "event");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, h.ev0, h.ev1), "event time");
    if (ms_out) *ms_out = ms;
    return ctrl[0];
}

std::string tune_key(const ldopf_batch& h) {
    hipDeviceProp_t prop{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    std::ostringstream k;
    k << prop.gcnArchName << "/cu" << prop.multiProcessorCount << "/S" << h.lp.S << "/N" << h.lp.gidx.size() << "/mf"
      << h.n_mf << "/vec" << h.n_vec << "/B" << h.B;
    return k.str();
}

bool read_tune_cache(const std::string& path, const std::string& key, int32_t* rows, int32_t* waves) {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        int32_t r, w;
        if (is >> k >> r >> w && k == key) {
            *rows = r;
            *waves = w;
            return true;
        }
    }
    return false;
}

void write_tune_cache(const std::string& path, const std::string& key, int32_t rows, int32_t waves) {
    std::ofstream f(path, std::ios::app);
    if (f) f << key << " " << rows << " " << waves << "\n";
}

}  // namespace

extern "C" {

int ldopf_batch_create(const ldopf_network* net, int32_t n_scen, const double* load_scale, const ldopf_options* opts,
                       void* stream, ldopf_batch** out) {
    return guard([&] {
        need(net, "net");
        need(out, "out");
        *out = nullptr;
        if (n_scen < 1 || n_scen > 1024) fail(LDOPF_INVALID_ARGUMENT, "n_scen must be in [1, 1024]");
        ldopf_options o;
        ldopf_default_options(&o);
        if (opts) o = *opts;
        check_options(o);
        check_batch_options(o);
        if (o.precision != LDOPF_FP32_MIXED)
            fail(LDOPF_UNSUPPORTED, "batched scenarios run in the FP32-mixed form (FP32 sweep, FP64 precompute and residuals)");
        ConsensusLP lp = assemble_network(*net);
        const int32_t nl = lp.n_load;
        std::vector<double> scale(size_t(n_scen) * std::max(nl, 1), 1.0);
        if (nl > 0) {
            need(load_scale, "load_scale");
            for (size_t i = 0; i < size_t(n_scen) * nl; ++i) {
                if (!std::isfinite(load_scale[i])) fail(LDOPF_INVALID_ARGUMENT, "non-finite load scale");
                scale[i] = load_scale[i];
            }
        }
        auto* h = new ldopf_batch();
        try {
            h->lp = std::move(lp);
            h->opts = o;
            h->B = n_scen;
            h->Bp = (n_scen + kTile - 1) / kTile * kTile;
            hip_check(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking), "stream");
            hip_check(hipEventCreate(&h->ev0), "event");
            hip_check(hipEventCreate(&h->ev1), "event");
            for (hipEvent_t& e : h->evc) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
            hip_check(hipHostMalloc(reinterpret_cast<void**>(&h->hctrl), 4 * sizeof(int64_t), hipHostMallocDefault),
                      "pinned control");
            if (stream) {
                // order after the caller's pending work
                hipEvent_t e;
                hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
                hip_check(hipEventRecord(e, static_cast<hipStream_t>(stream)), "event");
                hip_check(hipStreamWaitEvent(h->stream, e, 0), "event");
                (void)hipEventDestroy(e);
            }
            ConsensusLP& L = h->lp;
            hipStream_t s = h->stream;
            const int64_t S = L.S, nloc = int64_t(L.gidx.size());
            for (int32_t n : L.ns)
                if (n > 255) fail(LDOPF_UNSUPPORTED, "subsystems with more than 255 variables are not supported on the device");
            std::vector<int64_t> boff(S + 1, 0);
            for (int64_t i = 0; i < S; ++i) boff[i + 1] = boff[i] + int64_t(L.ns[i]) * L.ns[i];
            const int64_t words = boff[S];

            // device inputs of the precompute
            DevBuf<double> A, b, basis, abar, bbar, sc_d, tmp_basis, tmp_bbar;
            DevBuf<int32_t> ms, rank_d, flags_d, row_load, row_wcol, tmp_rank, tmp_bad, cls_d, vbrow_d, flag_d;
            DevBuf<int64_t> a_off, row_off, basis_off;
            A.upload(L.A, s, "upload A");
            b.upload(L.b, s, "upload b");
            h->ns.upload(L.ns, s, "upload n_s");
            ms.upload(L.ms, s, "upload m_s");
            a_off.upload(L.a_off, s, "upload offsets");
            row_off.upload(L.row_off, s, "upload offsets");
            h->loc_off.upload(L.loc_off, s, "upload offsets");
            basis_off.upload(boff, s, "upload offsets");
            row_load.upload(L.row_load, s, "upload load rows");
            row_wcol.upload(L.row_wcol, s, "upload load rows");
            sc_d.upload(scale, s, "upload load scale");
            basis.alloc(words, "basis");
            abar.alloc(words, "abar");
            bbar.alloc(nloc, "bbar");
            rank_d.alloc(S, "rank");
            flags_d.alloc(S, "flags");

            hip_check(hipEventRecord(h->ev0, s), "event");
            // unit-scale operators: ranks and the shared Abar of the MFMA class
            PrecomputeArgs pa{};
            pa.S = S;
            pa.ns = h->ns.p;
            pa.ms = ms.p;
            pa.a_off = a_off.p;
            pa.row_off = row_off.p;
            pa.loc_off = h->loc_off.p;
            pa.basis_off = basis_off.p;
            pa.A = A.p;
            pa.b = b.p;
            pa.basis = basis.p;
            pa.abar = abar.p;
            pa.bbar = bbar.p;
            pa.rank = rank_d.p;
            pa.flags = flags_d.p;
            pa.tol_dep = 1e-10;
            pa.tol_rhs = 1e-9;
            pa.max_n = *std::max_element(L.ns.begin(), L.ns.end());
            hip_check(launch_precompute(pa, s), "precompute");
            std::vector<int32_t> rank(S), flags(S);
            hip_check(hipMemcpyAsync(rank.data(), rank_d.p, S * 4, hipMemcpyDeviceToHost, s), "download ranks");
            hip_check(hipMemcpyAsync(flags.data(), flags_d.p, S * 4, hipMemcpyDeviceToHost, s), "download flags");
            hip_check(hipStreamSynchronize(s), "precompute");
            for (int64_t i = 0; i < S; ++i)
                if (flags[i]) fail(LDOPF_INCONSISTENT_SUBSYSTEM, "subsystem " + std::to_string(i) + " is inconsistent");

            // classes: shared operator (no load-scaled coefficient, n_s <= 64) -> MFMA
            std::vector<int32_t> cls(S, 0), vK(S, 0), vbrow(S, 0), vmode(S, 0);
            std::vector<int64_t> wofs(S, 0), ash_off_s(S, 0);
            std::vector<int32_t> mf, vec;
            int64_t wrows = 0, ash_words = 0;
            int32_t nmax = 1, kmax = 1;
            for (int64_t i = 0; i < S; ++i) {
                bool scaled = false;
                for (int64_t r = L.row_off[i]; r < L.row_off[i + 1]; ++r) {
                    const int32_t wc = L.row_wcol[r];
                    if (L.row_load[r] >= 0 && wc >= 0 &&
                        L.A[L.a_off[i] + (r - L.row_off[i]) * L.ns[i] + wc] != 0.0)
                        scaled = true;
                }
                const int32_t n = L.ns[i];
                nmax = std::max(nmax, n);
                // rank form for both classes: the K = min(r, n - r) rows of the
                // smaller of the row-space and complement bases
                const int32_t r = rank[i];
                vmode[i] = r <= n - r ? 1 : 0;
                vK[i] = std::min(r, n - r);
                vbrow[i] = vmode[i] ? 0 : r;
                kmax = std::max(kmax, vK[i]);
                if (!scaled) {
                    cls[i] = 0;
                    ash_off_s[i] = ash_words;
                    ash_words += int64_t(vK[i]) * n;
                    mf.push_back(int32_t(i));
                } else {
                    cls[i] = 1;
                    wofs[i] = wrows;
                    wrows += int64_t(vK[i]) * n;
                    vec.push_back(int32_t(i));
                }
            }
            h->n_mf = int64_t(mf.size());
            h->n_vec = int64_t(vec.size());
            // rows per wave of the local update: n_s <= 4 RPW
            if (nmax > 128) fail(LDOPF_UNSUPPORTED, "the batched path takes subsystems of at most 128 variables");
            h->nmax = nmax;
            h->kmax = kmax;
            h->rpw = nmax <= 40 ? 10 : (nmax <= 64 ? 16 : 32);
            {
                const size_t lds = local_lds(*h);
                if (lds > 65536)
                    hip_check(hipFuncSetAttribute(local_kernel(h->rpw), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)),
                              "local update LDS");
            }
            const int32_t Bp = h->Bp;
            // the local update indexes the global x with 32-bit offsets
            if (int64_t(L.n) * Bp >= (int64_t(1) << 31)) fail(LDOPF_UNSUPPORTED, "n x padded scenarios exceeds 2^31");
            h->BB.alloc(size_t(nloc) * Bp, "scenario bbar");
            h->W.alloc(size_t(std::max<int64_t>(wrows, 1)) * Bp, "scenario operators");
            h->w_words = wrows * Bp;
            h->cls.upload(cls, s, "upload classes");
            h->vK.upload(vK, s, "upload classes");
            vbrow_d.upload(vbrow, s, "upload classes");
            h->wofs.upload(wofs, s, "upload classes");
            flag_d.alloc(1, "flag");
            hip_check(hipMemsetAsync(flag_d.p, 0, 4, s), "flag");
            // zero the padded scenario columns of BB and W
            hip_check(hipMemsetAsync(h->BB.p, 0, h->BB.count * 4, s), "clear");
            hip_check(hipMemsetAsync(h->W.p, 0, h->W.count * 4, s), "clear");

            // per-scenario operators, in chunks of scenarios to bound the scratch
            const int64_t budget = int64_t(512) << 20;
            const int32_t C = int32_t(std::max<int64_t>(1, std::min<int64_t>(n_scen, budget / std::max<int64_t>(1, 8 * (words + nloc)))));
            tmp_basis.alloc(size_t(C) * words, "scratch");
            tmp_bbar.alloc(size_t(C) * nloc, "scratch");
            tmp_rank.alloc(size_t(C) * S, "scratch");
            tmp_bad.alloc(size_t(C) * S, "scratch");
            for (int32_t k0 = 0; k0 < n_scen; k0 += C) {
                const int32_t cn = std::min(C, n_scen - k0);
                PrecomputeBatchArgs pb{};
                pb.S = S;
                pb.nloc = nloc;
                pb.words = words;
                pb.k0 = k0;
                pb.C = cn;
                pb.n_load = nl;
                pb.ns = h->ns.p;
                pb.ms = ms.p;
                pb.a_off = a_off.p;
                pb.row_off = row_off.p;
                pb.loc_off = h->loc_off.p;
                pb.basis_off = basis_off.p;
                pb.A = A.p;
                pb.b = b.p;
                pb.row_load = row_load.p;
                pb.row_wcol = row_wcol.p;
                pb.scale = sc_d.p;
                pb.tmp_basis = tmp_basis.p;
                pb.tmp_bbar = tmp_bbar.p;
                pb.tmp_rank = tmp_rank.p;
                pb.tmp_bad = tmp_bad.p;
                pb.tol_dep = 1e-10;
                pb.tol_rhs = 1e-9;
                const unsigned grid = unsigned((S * cn + 3) / 4);
                hipLaunchKernelGGL(precompute_batch_kernel, dim3(grid), dim3(256), 0, s, pb);
                hip_check(hipGetLastError(), "batched precompute");
                PackArgs pk{};
                pk.S = S;
                pk.nloc = nloc;
                pk.words = words;
                pk.k0 = k0;
                pk.C = cn;
                pk.Bp = Bp;
                pk.ns = h->ns.p;
                pk.loc_off = h->loc_off.p;
                pk.basis_off = basis_off.p;
                pk.rank = rank_d.p;
                pk.cls = h->cls.p;
                pk.vK = h->vK.p;
                pk.vbrow = vbrow_d.p;
                pk.wofs = h->wofs.p;
                pk.tmp_basis = tmp_basis.p;
                pk.tmp_bbar = tmp_bbar.p;
                pk.tmp_rank = tmp_rank.p;
                pk.tmp_bad = tmp_bad.p;
                pk.BB = h->BB.p;
                pk.W = h->W.p;
                pk.flag = flag_d.p;
                hipLaunchKernelGGL(batch_pack_kernel, dim3(grid), dim3(256), 0, s, pk);
                hip_check(hipGetLastError(), "batched pack");
            }
            hip_check(hipEventRecord(h->ev1, s), "event");
            int32_t flag = 0;
            hip_check(hipMemcpyAsync(&flag, flag_d.p, 4, hipMemcpyDeviceToHost, s), "download flag");
            hip_check(hipStreamSynchronize(s), "batched precompute");
            float pms = 0.f;
            hip_check(hipEventElapsedTime(&pms, h->ev0, h->ev1), "event time");
            h->precompute_ms = pms;
            if (flag & 2) fail(LDOPF_INCONSISTENT_SUBSYSTEM, "a scaled subsystem has inconsistent rows");
            if (flag & 1) fail(LDOPF_UNSUPPORTED, "a subsystem's rank changes with the load scale");

            // shared FP32 rank-form rows of the MFMA class, from the unit-scale basis
            std::vector<double> basis_h(words);
            hip_check(hipMemcpy(basis_h.data(), basis.p, words * 8, hipMemcpyDeviceToHost), "download basis");
            std::vector<float> ash(std::max<int64_t>(ash_words, 1));
            for (int32_t i : mf) {
                const int64_t n = L.ns[i];
                for (int64_t k = 0; k < vK[i]; ++k)
                    for (int64_t j = 0; j < n; ++j)
                        ash[ash_off_s[i] + k * n + j] = float(basis_h[boff[i] + (vbrow[i] + k) * n + j]);
            }
            h->ash.upload(ash, s, "upload shared operators");
            std::vector<LocalMeta> meta(S);
            for (int64_t i = 0; i < S; ++i)
                meta[i] = LocalMeta{L.ns[i], cls[i], vK[i], vmode[i], L.loc_off[i], cls[i] ? wofs[i] : ash_off_s[i]};
            h->meta_h = std::move(meta);

            // consensus structure: copies of each variable, global data in FP32
            std::vector<int32_t> g32(nloc), var_off(L.n + 1, 0), var_copy(nloc);
            for (int64_t c = 0; c < nloc; ++c) {
                g32[c] = int32_t(L.gidx[c]);
                var_off[L.gidx[c] + 1]++;
            }
            for (int64_t v = 0; v < L.n; ++v) var_off[v + 1] += var_off[v];
            std::vector<int32_t> fill(var_off.begin(), var_off.end() - 1);
            for (int64_t c = 0; c < nloc; ++c) var_copy[fill[L.gidx[c]]++] = int32_t(c);
            std::vector<float> crho(L.n), lo(L.n), hi(L.n), invN(L.n);
            for (int64_t v = 0; v < L.n; ++v) {
                crho[v] = float(L.c[v] / o.rho);
                lo[v] = float(L.lo[v]);
                hi[v] = float(L.hi[v]);
                invN[v] = float(1.0 / double(var_off[v + 1] - var_off[v]));
            }
            h->gidx.upload(g32, s, "upload gidx");
            h->var_off.upload(var_off, s, "upload copies");
            h->var_copy.upload(var_copy, s, "upload copies");
            std::vector<int4> ell(L.n);
            for (int64_t v = 0; v < L.n; ++v) {
                int32_t e[4] = {-1, -1, -1, -1};
                for (int32_t i = 0; i < 4 && var_off[v] + i < var_off[v + 1]; ++i) e[i] = var_copy[var_off[v] + i];
                ell[v] = int4{e[0], e[1], e[2], e[3]};
            }
            h->ell.upload(ell, s, "upload copies");
            h->crho.upload(crho, s, "upload c");
            h->lo.upload(lo, s, "upload lo");
            h->hi.upload(hi, s, "upload hi");
            h->invN.upload(invN, s, "upload counts");
            h->x_init.upload(L.x_init, s, "upload start");
            h->X.alloc(2 * size_t(L.n) * Bp, "x");
            h->U.alloc(size_t(nloc) * Bp, "x_s - lambda / rho");
            h->LAM.alloc(size_t(nloc) * Bp, "lambda");
            h->active.alloc(Bp, "masks");
            h->conv.alloc(Bp, "masks");
            h->sflags.alloc(Bp, "masks");
            h->iters.alloc(Bp, "iterations");
            h->res.alloc(size_t(Bp) * 4, "residuals");
            h->ctrl.alloc(4, "control");
            h->part2.alloc(size_t(Bp / kTile) * kRedBlocks * 5 * kTile, "residual slices");
            h->tick.alloc(size_t(Bp / kTile), "reduction tickets");
            const int32_t rows = o.rows_per_part > 0 ? o.rows_per_part : 64;
            set_chunks(*h, rows, 256);
            batch_reset(*h);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

int ldopf_batch_destroy(ldopf_batch* h) {
    return guard([&] { delete h; });
}

int ldopf_batch_reset(ldopf_batch* h) {
    return guard([&] {
        need(h, "handle");
        batch_reset(*h);
    });
}

int ldopf_batch_solve(ldopf_batch* h, ldopf_batch_status* st) {
    return guard([&] {
        need(h, "handle");
        double ms = 0.0;
        const int64_t sweeps = run_to_done(*h, &ms);
        if (st) {
            std::memset(st, 0, sizeof(*st));
            std::vector<int32_t> conv(h->Bp), fl(h->Bp);
            hip_check(hipMemcpy(conv.data(), h->conv.p, h->Bp * 4, hipMemcpyDeviceToHost), "download masks");
            hip_check(hipMemcpy(fl.data(), h->sflags.p, h->Bp * 4, hipMemcpyDeviceToHost), "download masks");
            int32_t nc = 0, nbad = 0;
            for (int i = 0; i < h->B; ++i) {
                nc += conv[i] != 0;
                nbad += (fl[i] & 2) != 0;
            }
            st->sweeps = sweeps;
            st->n_scen = h->B;
            st->n_converged = nc;
            st->n_numerical = nbad;
            st->solve_ms = ms;
            st->precompute_ms = h->precompute_ms;
            st->code = nbad ? LDOPF_NUMERICAL : (h->opts.check_termination && nc < h->B ? LDOPF_NOT_CONVERGED : LDOPF_OK);
        }
    });
}

int ldopf_batch_get_scenario(const ldopf_batch* h, int32_t scen, ldopf_status* st) {
    return guard([&] {
        need(h, "handle");
        need(st, "status");
        if (scen < 0 || scen >= h->B) fail(LDOPF_INVALID_ARGUMENT, "scenario out of range");
        int64_t it = 0;
        int32_t conv = 0, fl = 0;
        double r[4];
        hip_check(hipMemcpy(&it, h->iters.p + scen, 8, hipMemcpyDeviceToHost), "download");
        hip_check(hipMemcpy(&conv, h->conv.p + scen, 4, hipMemcpyDeviceToHost), "download");
        hip_check(hipMemcpy(&fl, h->sflags.p + scen, 4, hipMemcpyDeviceToHost), "download");
        hip_check(hipMemcpy(r, h->res.p + 4 * int64_t(scen), 32, hipMemcpyDeviceToHost), "download");
        std::memset(st, 0, sizeof(*st));
        st->iterations = it;
        st->sweeps_computed = it;
        st->converged = conv;
        st->pres = r[0];
        st->dres = r[1];
        st->eps_prim = r[2];
        st->eps_dual = r[3];
        st->precompute_ms = h->precompute_ms;
        st->code = (fl & 2) ? LDOPF_NUMERICAL : (conv ? LDOPF_OK : LDOPF_NOT_CONVERGED);
    });
}

int ldopf_batch_get_global(const ldopf_batch* h, int32_t scen, double* x, int64_t cap) {
    return guard([&] {
        need(h, "handle");
        need(x, "x");
        if (scen < 0 || scen >= h->B) fail(LDOPF_INVALID_ARGUMENT, "scenario out of range");
        if (cap < h->lp.n) fail(LDOPF_BUFFER_TOO_SMALL, "x needs n entries");
        // x of the scenario's returned sweep: the half of its parity
        int64_t it = 0;
        hip_check(hipMemcpy(&it, h->iters.p + scen, 8, hipMemcpyDeviceToHost), "download");
        const float* xh = h->X.p + (it & 1) * h->lp.n * h->Bp;
        std::vector<float> col(h->lp.n);
        hip_check(hipMemcpy2D(col.data(), 4, xh + scen, size_t(h->Bp) * 4, 4, h->lp.n, hipMemcpyDeviceToHost), "download x");
        for (int64_t v = 0; v < h->lp.n; ++v) x[v] = col[v];
    });
}

int ldopf_batch_get_local(const ldopf_batch* h, int32_t scen, double* xs, double* lam, int64_t cap) {
    return guard([&] {
        need(h, "handle");
        if (scen < 0 || scen >= h->B) fail(LDOPF_INVALID_ARGUMENT, "scenario out of range");
        const int64_t nl = int64_t(h->lp.gidx.size());
        if (cap < nl) fail(LDOPF_BUFFER_TOO_SMALL, "x_s and lambda need N_loc entries");
        std::vector<float> u(nl), l(nl);
        hip_check(hipMemcpy2D(l.data(), 4, h->LAM.p + scen, size_t(h->Bp) * 4, 4, nl, hipMemcpyDeviceToHost), "download lambda");
        if (xs) {
            // x_s = u + lambda / rho, formed as the local update forms it
            hip_check(hipMemcpy2D(u.data(), 4, h->U.p + scen, size_t(h->Bp) * 4, 4, nl, hipMemcpyDeviceToHost), "download x_s");
            const float irho = float(1.0 / h->opts.rho);
            for (int64_t c = 0; c < nl; ++c) xs[c] = double(u[c] + l[c] * irho);
        }
        if (lam)
            for (int64_t c = 0; c < nl; ++c) lam[c] = l[c];
    });
}

int ldopf_batch_get_sizes(const ldopf_batch* h, ldopf_batch_sizes* o) {
    return guard([&] {
        need(h, "handle");
        need(o, "out");
        std::memset(o, 0, sizeof(*o));
        o->n = h->lp.n;
        o->n_sub = h->lp.S;
        o->n_local = int64_t(h->lp.gidx.size());
        o->n_scen = h->B;
        o->n_scen_padded = h->Bp;
        o->n_mfma_subsystems = h->n_mf;
        o->n_vector_subsystems = h->n_vec;
        o->scenario_operator_words = h->w_words;
        o->shared_operator_words = int64_t(h->ash.count);
        o->rows_per_chunk = h->rows_per_chunk;
        o->blocks_per_tile = h->grid;
        o->graph_sweeps = h->graph_sweeps;
    });
}

int ldopf_batch_tune(ldopf_batch* h, const char* cache_path, int32_t* rows_per_chunk, int32_t* blocks_per_tile) {
    return guard([&] {
        need(h, "handle");
        std::string path;
        if (cache_path) path = cache_path;
        const std::string key = tune_key(*h);
        int32_t best_r = h->rows_per_chunk, best_w = h->grid;
        if (path.empty() || !read_tune_cache(path, key, &best_r, &best_w)) {
            // time a short fixed number of sweeps for each candidate
            const int64_t keep_iter = h->opts.max_iter;
            const int32_t keep_check = h->opts.check_termination;
            h->opts.check_termination = 0;
            double best = 1e300;
            for (int32_t r : {32, 64, 128, 256})
                for (int32_t w : {64, 128, 256, 512}) {
                    set_chunks(*h, r, w);
                    // one untimed graph to warm up, then four timed ones
                    h->opts.max_iter = h->graph_sweeps;
                    drop_graph(*h);
                    batch_reset(*h);
                    run_to_done(*h, nullptr);
                    h->opts.max_iter = 4 * h->graph_sweeps;
                    drop_graph(*h);
                    batch_reset(*h);
                    double ms = 0.0;
                    run_to_done(*h, &ms);
                    if (ms < best) {
                        best = ms;
                        best_r = r;
                        best_w = w;
                    }
                }
            h->opts.max_iter = keep_iter;
            h->opts.check_termination = keep_check;
            drop_graph(*h);
            if (!path.empty()) write_tune_cache(path, key, best_r, best_w);
        }
        set_chunks(*h, best_r, best_w);
        batch_reset(*h);
        if (rows_per_chunk) *rows_per_chunk = best_r;
        if (blocks_per_tile) *blocks_per_tile = h->grid;
    });
}

int ldopf_batch_set_options(ldopf_batch* h, const ldopf_options* opts) {
    return guard([&] {
        need(h, "handle");
        need(opts, "opts");
        check_options(*opts);
        check_batch_options(*opts);
        if (opts->precision != h->opts.precision) fail(LDOPF_INVALID_ARGUMENT, "precision is fixed at creation");
        if (opts->rho != h->opts.rho) fail(LDOPF_INVALID_ARGUMENT, "rho is fixed at creation for a batch");
        h->opts = *opts;
        drop_graph(*h);
    });
}

}  // extern "C"
