// Device side of libldopf for gfx950 (CDNA4, wave64).
//
//  * precompute_kernel: once per network, FP64. For every subsystem, one wave
//    builds an orthonormal basis of R^{n_s} whose first rank_s rows span the
//    row space of A_s (modified Gram-Schmidt, two passes), completes it with
//    the orthogonal complement, and from it the operators of closed_2:
//    Abar_s = Q'Q - I (Q the row-space rows) and bbar_s = Q' beta, the
//    minimum-norm solution of A_s x = b_s. At full row rank these equal
//    A_s'(A_s A_s')^-1 A_s - I and A_s'(A_s A_s')^-1 b_s (Section III-B); a
//    dependent row is dropped after checking that its right-hand side is
//    consistent (the "row reduction" the paper asks for).
//
//  * sweep_kernel<T>: the ADMM loop of Algorithm 1 in one persistent,
//    cooperative launch. Each workgroup owns a run of subsystems and keeps
//    their operators (rank form), bbar, x_s and lambda in LDS for the whole
//    solve. One iteration: global update closed_1 for the variables the
//    workgroup touches, local update closed_2 in rank form, dual update
//    ADMM-3, residual partial sums in FP64, publication of the boundary
//    partial sums to the neighbouring workgroups, and the termination test
//    of Section III-C evaluated identically by every workgroup, three
//    sweeps later, by a wave of its own. There is no grid barrier: a
//    workgroup waits only for the exchange words it reads (boundary partial
//    sums of its neighbours; the residual sums, summed in two levels through
//    group leaders, of a sweep finished two sweeps earlier).
//
// The local update in rank form: with W the K_s rows of the smaller of the
// row-space basis (mode 1) and the complement basis (mode 0),
//   -Abar_s v = v - W'(W v)   (mode 1)   or   W'(W v)   (mode 0),
// so x_s = bbar_s - Abar_s (z + lambda / rho), the projection of
// z + lambda / rho onto {A_s x = b_s}, costs 2 K_s n_s instead of n_s^2.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "internal.h"
#include "layout.h"
#include "device.h"
#include "gs_core.h"

// Synchronisation words of the allocation-free solve (ldopf_solve_noalloc):
// every GPU the library runs on holds one copy until the process ends. Host
// code never passes this name to a kernel: it is a host-side stand-in, and
// the device address comes from hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) unsigned char scratch[ldopf::kStaticScratchBytes];

namespace ldopf {

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // once per device, with that device current: each GPU holds its own
        // copy of the array at its own address
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

namespace {

// DPP lane moves (gfx9 encodings): quad_perm [1,0,3,2] swaps neighbours,
// quad_perm [2,3,0,1] swaps pairs, row_half_mirror reverses each group of 8,
// row_mirror reverses each row of 16.
constexpr int kDppXor1 = 0xB1;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

// Every source lane of these patterns lies inside the row, so every lane is
// written and no fallback value is needed.
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of g lanes (g = 1, 2, 4, 8, 16); every lane of a
// group ends with the same bits. Needs every lane of the wave active.
template <typename T>
__device__ inline T group_sum(T v, int g) {
    if (g >= 2) v += dpp_move<kDppXor1>(v);
    if (g >= 4) v += dpp_move<kDppXor2>(v);
    if (g >= 8) v += dpp_move<kDppHalfMirror>(v);
    if (g >= 16) v += dpp_move<kDppMirror>(v);
    return v;
}

__device__ inline double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sums over each row of 16 lanes of five values (every lane of the row ends
// with the row's sums); the steps run across the five values so that their
// DPP chains overlap. Needs every lane of the wave active.
__device__ inline void row_sum5(double* v) {
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] += dpp_move<kDppXor1>(v[q]);
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] += dpp_move<kDppXor2>(v[q]);
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] += dpp_move<kDppHalfMirror>(v[q]);
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] += dpp_move<kDppMirror>(v[q]);
}

__device__ inline void st_agent(double* p, double v) {
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(float* p, float v) {
    __hip_atomic_store(reinterpret_cast<unsigned int*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

// ---------------------------------------------------------------------------
// Operator precompute (FP64). One wave per subsystem, lane l owns columns
// l, l + 64, ... (NQ of them: 4 for n_s <= 256, 16 for n_s <= 1024); the work
// row lives in registers, basis rows in global memory (each lane only
// touches its own columns).

template <int NQ>
__global__ __launch_bounds__(256) void precompute_kernel(PrecomputeArgs a) {
    __shared__ double sbeta[4][64 * NQ];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t s = int64_t(blockIdx.x) * 4 + wv;
    if (s >= a.S) return;
    int bad = 0;
    const int r = gs_project<NQ>(lane, a.ns[s], a.ms[s], a.A + a.a_off[s], a.b + a.row_off[s], nullptr, nullptr, nullptr,
                             a.tol_dep, a.tol_rhs, a.basis + a.basis_off[s], sbeta[wv], a.bbar + a.loc_off[s],
                             a.abar + a.basis_off[s], &bad);
    if (lane == 0) {
        a.rank[s] = r;
        a.flags[s] = bad;
    }
}

// ---------------------------------------------------------------------------
// Persistent sweep.

namespace {

struct SubLds {
    uint16_t row0, t0;
    uint16_t n, k;
    uint16_t mode, pad;
    uint32_t w0;
};
static_assert(sizeof(SubLds) == 16, "SubLds layout");

// Exchange words between workgroups. An empty word holds a signalling-NaN
// bit pattern: arithmetic only ever returns quiet NaNs, so a computed value
// never looks empty. A reader polls a word until it is not empty.
template <typename T>
struct Word;
template <>
struct Word<double> {
    using U = unsigned long long;
    static constexpr U kEmpty = 0x7FF4A5A5A5A5A5A5ull;
    __device__ static double value(U u) { return __longlong_as_double((long long)u); }
};
template <>
struct Word<float> {
    using U = unsigned int;
    static constexpr U kEmpty = 0x7FA5A5A5u;
    __device__ static float value(U u) { return __uint_as_float(u); }
};

template <typename T>
__device__ inline typename Word<T>::U ld_word(const T* p) {
    using U = typename Word<T>::U;
    return __hip_atomic_load(reinterpret_cast<U*>(const_cast<T*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_empty(T* p) {
    using U = typename Word<T>::U;
    __hip_atomic_store(reinterpret_cast<U*>(p), Word<T>::kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Re-read an exchange word until it is written; a wait longer than `limit`
// wall-clock ticks clears *ok (a broken launch then ends instead of hanging).
template <typename T>
__device__ inline T await_word(const T* p, typename Word<T>::U u, uint64_t limit, int* ok) {
    if (u != Word<T>::kEmpty) return Word<T>::value(u);
    const uint64_t t0 = wall_clock64();
    // re-read back to back; the clock (a scalar memory read) only every
    // 16th time, so that a word is seen about one load after it lands
    for (uint32_t n = 1;; ++n) {
        u = ld_word(p);
        if (u != Word<T>::kEmpty) return Word<T>::value(u);
        if ((n & 15u) == 0 && wall_clock64() - t0 > limit) {
            *ok = 0;
            return T(0);
        }
    }
}

// Lanes per (subsystem, basis row) task of t = W v: as many as the
// workgroup can give, up to 8, so that long rows do not serialize.
__device__ inline int task_lanes(int tasks, int threads) {
    int g = 1;
    while (g < 8 && tasks * g * 2 <= threads) g <<= 1;
    return g;
}

}  // namespace

// A workgroup-uniform 32-bit value kept in a vector register: LDS addresses
// are formed in vector registers in any case, while the scalar register file
// is the one this kernel runs short of.
__device__ inline uint32_t in_vgpr(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ inline double in_vgpr(double x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ inline float in_vgpr(float x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Compile-time variants of the sweep: bit 0 per-phase profiling, bit 1 the
// aggregated residual form, bit 2 residual balancing of rho (without it rho
// is a constant of the launch).
constexpr int kModeProf = 1, kModeAgg = 2, kModeRho = 4;

// One workgroup's whole solve: part `part` of the problem `a` describes.
template <typename T, int MODE>
__device__ __attribute__((always_inline)) inline void sweep_body(const SweepArgs<T>& a, const unsigned part) {
    constexpr bool PROF = (MODE & kModeProf) != 0, AGG = (MODE & kModeAgg) != 0, RHO = (MODE & kModeRho) != 0;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int ok_lds;
    __shared__ int test_lds;  // 1 stop, 2 converged, 4 non-finite: the last test
    __shared__ double rho_of[8];  // rho of sweep k in entry k % 8 (residual balancing)
    // the rule's parameters, read only where it is evaluated (kept out of
    // the scalar registers, the scarce file of this kernel)
    __shared__ double rule_mu, rule_tau;
    __shared__ int rule_period, rule_max;
    __shared__ double* rule_log;
    // the problem's own workgroup size; in a launch of several problems the
    // waves beyond it end here (a barrier waits only for running waves), so
    // every problem runs exactly as in a launch of its own
    const int tid = threadIdx.x, nt = a.block, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
    if (tid >= nt) return;
    const PartInfo pi = a.parts[part];
    const LdsLayout L = lds_layout(sizeof(T), uint32_t(pi.w_words), uint32_t(pi.n_row), uint32_t(pi.n_tk),
                                   uint32_t(pi.n_var), uint32_t(pi.n_sub), uint32_t(nw));
    T* W = reinterpret_cast<T*>(smem + in_vgpr(L.W));
    T* bbar = reinterpret_cast<T*>(smem + in_vgpr(L.bbar));
    // state buffers, selected by offset from the shared base so that every
    // access stays an LDS access (a table of pointers would not)
    const uint32_t s_xs = in_vgpr(L.xs[1] - L.xs[0]), s_lam = in_vgpr(L.lam[1] - L.lam[0]), s_xl = in_vgpr(L.xloc[1] - L.xloc[0]);
    const uint32_t o_xs = in_vgpr(L.xs[0]), o_lam = in_vgpr(L.lam[0]), o_xl = in_vgpr(L.xloc[0]);
    auto XS = [&](int b) { return reinterpret_cast<T*>(smem + o_xs + uint32_t(b) * s_xs); };
    auto LAM = [&](int b) { return reinterpret_cast<T*>(smem + o_lam + uint32_t(b) * s_lam); };
    auto XL = [&](int b) { return reinterpret_cast<T*>(smem + o_xl + uint32_t(b) * s_xl); };
    T* vb = reinterpret_cast<T*>(smem + in_vgpr(L.v));
    T* tb = reinterpret_cast<T*>(smem + in_vgpr(L.t));
    T* ownp = reinterpret_cast<T*>(smem + in_vgpr(L.ownp));
    T* cvar = reinterpret_cast<T*>(smem + in_vgpr(L.crho));  // c of each variable
    T* vlo = reinterpret_cast<T*>(smem + in_vgpr(L.lo));
    T* vhi = reinterpret_cast<T*>(smem + in_vgpr(L.hi));
    T* vcnt = reinterpret_cast<T*>(smem + in_vgpr(L.cnt));
    int32_t* sbase = reinterpret_cast<int32_t*>(smem + in_vgpr(L.slot_lo));
    int32_t* sm_ = reinterpret_cast<int32_t*>(smem + in_vgpr(L.slot_hi));
    int32_t* sme = reinterpret_cast<int32_t*>(smem + in_vgpr(L.slot_own));
    uint16_t* rlv = reinterpret_cast<uint16_t*>(smem + in_vgpr(L.row_lvar));
    uint16_t* rsub = reinterpret_cast<uint16_t*>(smem + in_vgpr(L.row_sub));
    uint16_t* coff = reinterpret_cast<uint16_t*>(smem + in_vgpr(L.copy_off));
    uint16_t* crow = reinterpret_cast<uint16_t*>(smem + in_vgpr(L.copy_rows));
    uint16_t* tks = reinterpret_cast<uint16_t*>(smem + in_vgpr(L.tk_sub));
    SubLds* meta = reinterpret_cast<SubLds*>(smem + in_vgpr(L.meta));
    uint2* tkm = reinterpret_cast<uint2*>(smem + in_vgpr(L.tk_m));
    uint2* rwm = reinterpret_cast<uint2*>(smem + in_vgpr(L.row_m));
    uint16_t* vr0 = reinterpret_cast<uint16_t*>(smem + in_vgpr(L.var_r0));
    double* red = reinterpret_cast<double*>(smem + in_vgpr(L.red));
    double* aggw = reinterpret_cast<double*>(smem + in_vgpr(L.agg));
    double* tot = red + 32 * nw;  // after the row sums [waves][4][8]

    // rho of the sweep being computed (sweep done + 1) and 1/rho of the next
    // one, whose global update the partial sums published in this sweep feed
    // (they differ only where residual balancing changes rho)
    double rho_c = RHO ? in_vgpr(a.rho) : a.rho;
    T rho_cT = RHO ? in_vgpr(T(a.rho)) : T(a.rho);
    T irho_c = RHO ? in_vgpr(T(1.0 / a.rho)) : T(1.0 / a.rho), irho_n = irho_c;
    const int R = pi.n_row, V = pi.n_var, TK = pi.n_tk;
    const unsigned P = unsigned(a.P);
    const int64_t ns = a.n_slots;
    const uint64_t limit = a.spin_limit;

    // ---- load this part into LDS
    if (tid == 0) ok_lds = 1;
    if (RHO && tid < 8) rho_of[tid] = a.rho;
    if (RHO && tid == 0) {
        rule_mu = a.rho_mu;
        rule_tau = a.rho_tau;
        rule_period = a.rho_update ? a.rho_period : 0;
        rule_max = a.rho_update ? a.rho_max_changes : 0;
        rule_log = a.rho_log;
    }
    for (int i = tid; i < pi.n_sub; i += nt) {
        const SubMeta m = a.subs[pi.sub_begin + i];
        meta[i] = SubLds{m.row0, m.t0, m.n, m.k, m.mode, 0, m.w0};
    }
    for (int r = tid; r < R; r += nt) {
        const int canon = a.row_canon[pi.row_begin + r];
        bbar[r] = T(a.bbar[canon]);
        XS(0)[r] = T(a.xs[canon]);
        LAM(0)[r] = T(a.lam[canon]);
        rlv[r] = a.row_lvar[pi.row_begin + r];
        rsub[r] = a.row_sub[pi.row_begin + r];
        crow[r] = a.var_copy_rows[pi.copy_begin + r];
    }
    for (int v = tid; v <= V; v += nt) coff[v] = a.var_copy_off[pi.coff_begin + v];
    for (int v = tid; v < V; v += nt) {
        const int g = a.var_gid[pi.var_begin + v];
        cvar[v] = T(a.c[g]);
        vlo[v] = T(a.lo[g]);
        vhi[v] = T(a.hi[g]);
        vcnt[v] = T(1.0 / a.cnt[g]);  // reciprocal of the copy count N_i
        sbase[v] = a.var_slot_lo[pi.var_begin + v];
        sm_[v] = a.var_slot_hi[pi.var_begin + v];
        sme[v] = a.var_slot[pi.var_begin + v];
    }
    for (int q = tid; q < TK; q += nt) tks[q] = a.tk_sub[pi.tk_begin + q];
    __syncthreads();
    // each task's and each row's operator offsets in one word, so that the
    // phases reach their operands with one LDS read instead of two
    // (operator words, rows and tasks of a part all stay below 2^16)
    for (int q = tid; q < TK; q += nt) {
        const SubLds m = meta[tks[q]];
        tkm[q] = make_uint2((m.w0 + uint32_t(q - m.t0) * m.n) | (uint32_t(m.row0) << 16), m.n);
    }
    for (int v = tid; v < V; v += nt) vr0[v] = crow[coff[v]];
    for (int r = tid; r < R; r += nt) {
        const SubLds m = meta[rsub[r]];
        rwm[r] = make_uint2((m.w0 + uint32_t(r - m.row0)) | (uint32_t(m.t0) << 16),
                            uint32_t(m.n) | (uint32_t(m.k) << 12) | (uint32_t(m.mode) << 24));
    }
    for (int i = wv; i < pi.n_sub; i += nw) {
        const SubMeta m = a.subs[pi.sub_begin + i];
        const int kn = int(m.k) * int(m.n);
        for (int q = lane; q < kn; q += 64) {
            const int k = q / m.n, j = q - k * m.n;
            W[m.w0 + q] = T(a.basis[m.basis + uint64_t(m.brow + k) * m.n + j]);
        }
    }
    __syncthreads();

    // The last wave reads the residual sums of all parts back and runs the
    // test (during the global update); it holds no rows and takes
    // no part in the global update and the boundary exchange, whose loads
    // would otherwise wait (in-order vmcnt) on its loads in flight. The other
    // waves leave it their residual sums per row of 16 lanes.
    const int tw = nw - 1;
    const int g_threads = nt - 64;  // two waves at least (checked by the host)
    const int n_work = g_threads >> 6;  // waves that hold rows

    // publish a boundary variable's partial sum to every other owner
    auto publish = [&](T* buf, int v, T acc) {
        const int sb = sbase[v];
        if (sb < 0) return;
        const int m = sm_[v], me = sme[v];
        for (int j = 0; j < m; ++j)
            if (j != me) st_agent(buf + sb + j * m + me, acc);
    };
    // the words addressed to this part for a boundary variable (up to four
    // loads in flight)
    auto prefetch = [&](const T* buf, int v, typename Word<T>::U* u) {
        const int sb = sbase[v], m = sm_[v], me = sme[v];
        const int f = m - 1;
        const T* rd = buf + sb + me * m;
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = k < f ? ld_word(rd + (k < me ? k : k + 1)) : Word<T>::kEmpty;
    };
    // all owners' partial sums in owner order: the m - 1 foreign ones
    // waited for (re-read while empty) and their words emptied
    auto gather = [&](T* buf, int v) -> T {
        const int sb = sbase[v], m = sm_[v], me = sme[v];
        const int f = m - 1;
        const T* rd = buf + sb + me * m;
        typename Word<T>::U u[4];
        prefetch(buf, v, u);
        T w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = k < f ? await_word(rd + (k < me ? k : k + 1), u[k], limit, &ok_lds) : T(0);
        T s = T(0);
        for (int i = 0; i < m; ++i) {
            T val;
            if (i == me) {
                val = ownp[v];
            } else {
                const int k = i < me ? i : i - 1;
                if (k < 4) {
                    val = k == 0 ? w[0] : (k == 1 ? w[1] : (k == 2 ? w[2] : w[3]));
                } else {
                    val = await_word(rd + i, ld_word(rd + i), limit, &ok_lds);
                }
                st_empty(buf + sb + me * m + i);
            }
            s = i == 0 ? val : s + val;
        }
        return s;
    };
    // Aggregated residual form: a boundary variable's per-owner sums of
    // rho (x_k - x_k_prev) and of lambda_k over its copies go to its first
    // owner (owner index 0), which adds the m sums in owner order, squares
    // the two totals and empties the words. Words: [parity][quantity][slot],
    // the slot of (reader 0, writer me) = slot base + me.
    auto agg_publish = [&](int par, int v, double dsum, double lsum) {
        double* w0 = a.bagg + int64_t(par) * 2 * ns + sbase[v] + sme[v];
        st_agent(w0, dsum);
        st_agent(w0 + ns, lsum);
    };
    auto agg_collect = [&](int par, int v, double* d2, double* l2) {
        double* w0 = a.bagg + int64_t(par) * 2 * ns + sbase[v];
        const int m = sm_[v];
        double ds = 0.0, ls = 0.0;
        for (int j = 0; j < m; ++j) {
            const double dj = await_word(w0 + j, ld_word(w0 + j), limit, &ok_lds);
            const double lj = await_word(w0 + ns + j, ld_word(w0 + ns + j), limit, &ok_lds);
            st_empty(w0 + j);
            st_empty(w0 + ns + j);
            ds = j == 0 ? dj : ds + dj;
            ls = j == 0 ? lj : ls + lj;
        }
        *d2 += ds * ds;
        *l2 += ls * ls;
    };
    // one wave's aggregated sums into LDS for the test wave (every lane active)
    auto agg_to_lds = [&](double d2, double l2) {
        d2 = group_sum(d2, 16);
        l2 = group_sum(l2, 16);
        d2 = read_lane(d2, 0) + read_lane(d2, 16) + read_lane(d2, 32) + read_lane(d2, 48);
        l2 = read_lane(l2, 0) + read_lane(l2, 16) + read_lane(l2, 32) + read_lane(l2, 48);
        if (lane == 0) {
            aggw[wv * 2] = d2;
            aggw[wv * 2 + 1] = l2;
        }
    };
    // interior variables' aggregated sums of the last published sweep, carried
    // by the thread that owns them from the publication to the next global update
    double agg_d2 = 0.0, agg_l2 = 0.0;

    // ---- partial sums of the starting state for the first global update
    for (int v = tid; tid < g_threads && v < V; v += g_threads) {
        T acc = T(0);
        for (int q = coff[v]; q < coff[v + 1]; ++q) {
            const int r = crow[q];
            acc += XS(0)[r] - LAM(0)[r] * irho_c;
        }
        ownp[v] = acc;
        publish(a.bpart, v, acc);
    }
    __syncthreads();

    const int GA = task_lanes(TK, g_threads);
    const int lgGA = GA == 8 ? 3 : (GA == 4 ? 2 : (GA == 2 ? 1 : 0));  // GA is a power of two
    // Residual sums, reduced in two levels by wave tw. Level 1: every part's
    // 5 sums of a sweep (ring entry [8][P], quantity-major), read only by its
    // group leader, the first of each kGroup consecutive parts, which adds
    // its members' sums and publishes them (level 2, ring entry [8][kGroup]);
    // every part then reads the group sums and runs the test. Lanes hold the
    // five quantities transposed: lane 16q + i holds quantity q (q < 4) of
    // member (group) i in word A, and lanes i < 16 hold quantity 4 in word B,
    // so that two 16-lane sums serve all five. Every part adds in the same
    // lane order, so every part takes the same decision.
    static_assert(kGroup == 16, "one lane row per group");
    const bool leader = part % kGroup == 0;
    const unsigned grp = part / kGroup, ngroups = (P + kGroup - 1) / kGroup;
    // word B holds quantity 4 (lanes < 16) and, in the aggregated form, the
    // aggregated dual residual and dual norm (quantities 5, 6; lanes 16..47)
    constexpr int nqb = AGG ? 3 : 1, nq = 4 + nqb;
    const int qa = lane >> 4, gi = lane & 15, qb = 4 + qa;
    const unsigned member = part + unsigned(gi);
    const bool mem_a = member < P, mem_b = mem_a && qa < nqb;
    const bool grp_a = unsigned(gi) < ngroups, grp_b = grp_a && qa < nqb;
    unsigned long long w1a = 0, w1b = 0, w2a = 0, w2b = 0;
    auto ring1 = [&](int64_t sweep) -> double* { return a.rpart + int64_t(sweep & (kRing - 1)) * P * 8; };
    auto ring2 = [&](int64_t sweep) -> double* { return a.gpart + int64_t(sweep & (kRing - 1)) * 8 * kGroup; };
    auto issue_members = [&](int64_t sweep) {
        const double* base = ring1(sweep) + member;
        w1a = mem_a ? ld_word(base + qa * P) : 0ull;
        w1b = mem_b ? ld_word(base + qb * P) : 0ull;
    };
    auto issue_groups = [&](int64_t sweep) {
        const double* base = ring2(sweep) + gi;
        w2a = grp_a ? ld_word(base + qa * kGroup) : 0ull;
        w2b = grp_b ? ld_word(base + qb * kGroup) : 0ull;
    };
    // leader: its members' sums of `sweep` added and published; the members'
    // words emptied (the leader is their only reader)
    auto group_sums = [&](int64_t sweep) {
        double* base = ring1(sweep) + member;
        double va = mem_a ? await_word(base + qa * P, w1a, limit, &ok_lds) : 0.0;
        double vb = mem_b ? await_word(base + qb * P, w1b, limit, &ok_lds) : 0.0;
        va = group_sum(va, kGroup);
        vb = group_sum(vb, kGroup);
        double* g = ring2(sweep) + grp;
        if (gi == 0) st_agent(g + qa * kGroup, va);
        if (gi == 0 && qa < nqb) st_agent(g + qb * kGroup, vb);
        if (mem_a) st_empty(base + qa * P);
        if (mem_b) st_empty(base + qb * P);
    };
    uint64_t tprof[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t tw_prof = 0;  // wave tw's time in the test's totals, inside phase 0
    uint64_t tlast = 0;
    auto stamp = [&](int ph) {
        if (PROF && tid == 0) {
            const uint64_t now = wall_clock64();
            tprof[ph] += now - tlast;
            tlast = now;
        }
    };
    if (PROF && tid == 0) tlast = wall_clock64();

    int64_t done = 0;     // sweeps computed
    int64_t result = 0;   // sweep whose state is returned
    int converged = 0, nonfinite = 0;
    bool ok = true;
    double d[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double sq = sqrt(double(a.nloc));
    // dimension of the dual residual's vector: every copy, or (aggregated
    // form) every global variable
    const double sqd = AGG ? sqrt(double(a.n)) : sq;
    // residual balancing, kept by lane 0 of wave tw: rho of the latest sweep
    // scheduled so far, and the changes decided
    double rho_sched = a.rho;
    int64_t rho_changes = 0;
    // termination test of one finished sweep; identical on every workgroup
    // wave tw: the grid-wide sums of one sweep from the group sums (loads
    // issued by issue_groups), into LDS for every thread. With may_change,
    // also the residual-balancing rule for that sweep (same sums, hence the
    // same decision on every workgroup).
    auto totals = [&](int64_t sweep, bool may_change) {
        const double* base = ring2(sweep) + gi;
        double va = grp_a ? await_word(base + qa * kGroup, w2a, limit, &ok_lds) : 0.0;
        double vb = grp_b ? await_word(base + qb * kGroup, w2b, limit, &ok_lds) : 0.0;
        va = group_sum(va, kGroup);
        vb = group_sum(vb, kGroup);
        // the grid totals: quantity q < 4 in lane 16q of A, quantity 4 + q
        // in lane 16q of B; their square roots taken lane-parallel
        if (gi == 0) tot[qa] = va;
        if (gi == 0 && qa < nqb) tot[qb] = vb;
        const double ra = sqrt(va), rb = sqrt(vb);
        const double r0 = read_lane(ra, 0), r1 = read_lane(ra, 16), r2 = read_lane(ra, 32), r3 = read_lane(ra, 48);
        const double r4 = read_lane(rb, 0);
        const double r5 = AGG ? read_lane(rb, 16) : 0.0, r6 = AGG ? read_lane(rb, 32) : 0.0;
        // the test itself, once per workgroup (lane 0 of wave tw); the sums
        // are of squares, so a non-finite sum shows in its square root (the
        // dual residual sums are of rho (x_s - x_s_prev), rho of that sweep)
        if (lane == 0) {
            const double pres = r0, dres = AGG ? r5 : r1;
            const double eps_p = sq * a.eps_abs + a.eps_rel * fmax(r2, r3);
            const double eps_d = sqd * a.eps_abs + a.eps_rel * (AGG ? r6 : r4);
            const int nf = !isfinite(r0 + r1 + r2 + r3 + r4 + r5 + r6);
            const int cv = pres <= eps_p && dres <= eps_d;
            const int stop = nf || (a.check && cv);
            test_lds = (stop ? 1 : 0) | (cv ? 2 : 0) | (nf ? 4 : 0);
            const int period = rule_period;
            if (RHO && may_change && !stop && period > 0 && sweep % period == 0 && rho_changes < rule_max && eps_p > 0.0 &&
                eps_d > 0.0) {
                const double rr = pres / eps_p, ss = dres / eps_d, mu = rule_mu, tau = rule_tau;
                const double f = rr > mu * ss ? tau : (ss > mu * rr ? 1.0 / tau : 1.0);
                if (f != 1.0) {
                    rho_sched *= f;
                    if (part == 0) {
                        double* lg = rule_log;
                        lg[2 * rho_changes] = double(sweep + kRhoLag);
                        lg[2 * rho_changes + 1] = rho_sched;
                    }
                    ++rho_changes;
                }
            }
            if (part == 0 && sweep <= a.hist_cap && ok_lds) {
                double* h = a.hist + (sweep - 1) * 4;
                h[0] = pres;
                h[1] = dres;
                h[2] = eps_p;
                h[3] = eps_d;
            }
        }
    };
    // the outcome of that test, for every thread (after a block barrier)
    auto decide = [&]() -> bool {
        ok = ok_lds != 0;
        const int f = test_lds;
        converged = (f & 2) != 0;
        nonfinite = (f & 4) != 0;
        return (f & 1) != 0;
    };

    bool stopped = false;
    // The two roles run loops of their own (so that neither carries the
    // other's registers), with the same barriers in the same order: B1 after
    // the global update (where both read the outcome of the test), B2 after
    // the gather, B3 after t = W v, B4 after the local update.
    if (wv == tw) {
        while (done < a.max_iter) {
            // the test of sweep done - 2, during the global update
            if (done >= 3) {
                const uint64_t t0 = PROF ? wall_clock64() : 0;
                totals(done - 2, true);
                if (PROF && lane == 0) tw_prof += wall_clock64() - t0;
                // every part has read the group sums of sweep done - 5: their
                // sums of sweep done - 2 are all in, and each part tests
                // sweep j before it publishes sweep j + 3
                if (leader && lane < nq && done >= 6) st_empty(ring2(done - 5) + lane * kGroup + grp);
            }
            // rho of sweep done + 2 (a change decided from the test of sweep
            // done - 2), read by the row waves after B1
            if (RHO && lane == 0) rho_of[(done + 2) & 7] = rho_sched;
            __syncthreads();  // B1
            if (ok_lds == 0) {
                ok = false;
                break;
            }
            if (done >= 3 && decide()) {
                result = done - 2;
                stopped = true;
                break;
            }
            if (AGG && done >= 1) {
                // this part's aggregated sums of sweep done (completed by the
                // row waves' global update) beside its other sums of that sweep
                if (lane < 2) {
                    double q = 0.0;
                    for (int w = 0; w < n_work; ++w) q += aggw[w * 2 + lane];
                    st_agent(ring1(done) + (5 + lane) * P + part, q);
                }
            }
            __syncthreads();  // B2
            // its stores of the last phase complete first (issued a phase or
            // more ago); then the loads of this sweep: the leader's members'
            // sums of the previous sweep, and the group sums of sweep
            // done - 1 for the next test
            __builtin_amdgcn_s_waitcnt(0);
            if (leader && done >= 1) issue_members(done);
            if (done >= 2) issue_groups(done - 1);
            __syncthreads();  // B3
            __syncthreads();  // B4
            // its loads of the t phase have long returned: waiting for them
            // here, before any store of this phase, keeps the later waits on
            // them (group sums, totals) from also waiting for those stores
            __builtin_amdgcn_s_waitcnt(0);
            // group-sum words of sweep done - 1 that were still empty when
            // loaded in the t phase are loaded again, before this phase's
            // stores (the wait above made their values known)
            if (done >= 2) {
                const double* base = ring2(done - 1) + gi;
                if (grp_a && w2a == Word<double>::kEmpty) w2a = ld_word(base + qa * kGroup);
                if (grp_b && w2b == Word<double>::kEmpty) w2b = ld_word(base + qb * kGroup);
            }
            // this part's sums of the sweep from the row sums of the work
            // waves: lane 8q + j adds rows j, j + 8, ... of quantity q, then
            // the 8 lanes of q are added
            double sq_ = 0.0;
            if (lane < 40) {
                const int q = lane >> 3;
                for (int i = lane & 7; i < 4 * n_work; i += 8) sq_ += red[i * 8 + q];
            }
            sq_ = group_sum(sq_, 8);
            if (leader && done >= 1) group_sums(done);
            if (lane < 40 && (lane & 7) == 0) st_agent(ring1(done + 1) + (lane >> 3) * P + part, sq_);
            ++done;
        }
    } else {
        int cur = 0;  // x_s, lambda buffer of sweep `done` (sweep k lives in buffer k % 3, its x in k % 4)
        while (done < a.max_iter) {
            const int nx = cur == 2 ? 0 : cur + 1;
            const int bp = int(done & 1);  // exchange-word parity
            T* bcur = a.bpart + int64_t(bp) * ns;
            T* bnx = a.bpart + int64_t(bp ^ 1) * ns;
            T* xg = XL(int((done + 1) & 3));
            // closed_1: clipped average of the copies; in the aggregated
            // form, owner 0 of each boundary variable also completes the
            // aggregated sums of sweep done
            double ad2 = agg_d2, al2 = agg_l2;
            for (int v = tid; v < V; v += g_threads) {
                const T s = sbase[v] < 0 ? ownp[v] : gather(bcur, v);
                if (AGG && done >= 1 && sbase[v] >= 0 && sme[v] == 0) agg_collect(bp, v, &ad2, &al2);
                T xv = (s - cvar[v] * irho_c) * vcnt[v];
                xv = xv < vlo[v] ? vlo[v] : xv;
                xv = xv > vhi[v] ? vhi[v] : xv;
                xg[v] = xv;
            }
            if (AGG && done >= 1) agg_to_lds(ad2, al2);
            if (PROF && tid == 0) tprof[7] += wall_clock64() - tlast;  // the workgroup's own global update, inside phase 0
            __syncthreads();  // B1
            if (ok_lds == 0) {
                ok = false;
                break;
            }
            if (done >= 3 && decide()) {
                // x_s, lambda of sweep done - 2 are intact (this sweep's
                // local update has not run), and so is its x (buffer % 4)
                result = done - 2;
                stopped = true;
                break;
            }
            // rho of the next sweep, whose global update this sweep's
            // published partial sums feed
            const double rho_n = RHO ? in_vgpr(rho_of[(done + 2) & 7]) : a.rho;
            if (RHO) irho_n = in_vgpr(T(1.0 / rho_n));
            stamp(0);
            // v = B_s x + lambda_s / rho
            const T* lc = LAM(cur);
            for (int r = tid; r < R; r += g_threads) vb[r] = xg[rlv[r]] + lc[r] * irho_c;
            __syncthreads();  // B2
            stamp(1);
            // t = W v: GA lanes per (subsystem, basis row) task, then a lane-group sum
            for (int base = 0; base < TK * GA; base += g_threads) {
                const int q0 = base + tid;
                const int task = q0 >> lgGA, sub = q0 & (GA - 1);
                T acc = T(0);
                if (task < TK) {
                    const uint2 tm = tkm[task];
                    const T* wr = W + (tm.x & 0xffffu);
                    const T* vv = vb + (tm.x >> 16);
                    const int n_t = int(tm.y);
                    // four products per step, their eight loads issued together
                    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
                    int j = sub;
                    for (; j + 3 * GA < n_t; j += 4 * GA) {
                        const T w0 = wr[j], w1 = wr[j + GA], w2 = wr[j + 2 * GA], w3 = wr[j + 3 * GA];
                        const T v0 = vv[j], v1 = vv[j + GA], v2 = vv[j + 2 * GA], v3 = vv[j + 3 * GA];
                        a0 += w0 * v0;
                        a1 += w1 * v1;
                        a2 += w2 * v2;
                        a3 += w3 * v3;
                    }
                    for (; j < n_t; j += GA) a0 += wr[j] * vv[j];
                    acc = (a0 + a1) + (a2 + a3);
                }
                acc = group_sum(acc, GA);
                if (task < TK && sub == 0) tb[task] = acc;
            }
            __syncthreads();  // B3
            stamp(2);
            // closed_2 in rank form, then ADMM-3; residual sums in FP64
            const T* xc = XS(cur);
            T* xn = XS(nx);
            T* ln = LAM(nx);
            {
                double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, p4 = 0.0;
                for (int r = tid; r < R; r += g_threads) {
                    const uint2 rm = rwm[r];
                    const T* wc = W + (rm.x & 0xffffu);
                    const T* tt = tb + (rm.x >> 16);
                    // four products per step, their eight loads issued together
                    const int n_ = int(rm.y & 0xfffu), K_ = int((rm.y >> 12) & 0xfffu);
                    const bool mode1 = ((rm.y >> 24) & 1u) != 0;
                    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
                    int k = 0;
                    for (; k + 4 <= K_; k += 4) {
                        const T w0 = wc[k * n_], w1 = wc[(k + 1) * n_], w2 = wc[(k + 2) * n_], w3 = wc[(k + 3) * n_];
                        const T t0 = tt[k], t1 = tt[k + 1], t2 = tt[k + 2], t3 = tt[k + 3];
                        a0 += w0 * t0;
                        a1 += w1 * t1;
                        a2 += w2 * t2;
                        a3 += w3 * t3;
                    }
                    for (; k < K_; ++k) a0 += wc[k * n_] * tt[k];
                    const T acc = (a0 + a1) + (a2 + a3);
                    const T vr = vb[r];
                    const T y = mode1 ? bbar[r] + (vr - acc) : bbar[r] + acc;
                    const T z = xg[rlv[r]];
                    const T lnew = lc[r] + rho_cT * (z - y);
                    xn[r] = y;
                    ln[r] = lnew;
                    const double dz = double(z) - double(y);
                    const double dx = rho_c * (double(y) - double(xc[r]));
                    p0 += dz * dz;
                    p1 += dx * dx;
                    p2 += double(z) * double(z);
                    p3 += double(y) * double(y);
                    p4 += double(lnew) * double(lnew);
                }
                // each row of 16 lanes sums its values; its first lane leaves
                // them for wave tw
                double pq[5] = {p0, p1, p2, p3, p4};
                row_sum5(pq);
                if ((lane & 15) == 0) {
                    double* o = red + (wv * 4 + (lane >> 4)) * 8;
#pragma unroll
                    for (int q = 0; q < 5; ++q) o[q] = pq[q];
                }
                // this sweep's emptied exchange words are stored before any
                // partial sum of this sweep is published
                __builtin_amdgcn_s_waitcnt(0);
            }
            __syncthreads();  // B4
            stamp(3);
            // partial sums for the next global update; publish boundary slots
            // (every variable has a copy in the part; its first copy's row
            // is read beside the copy range)
            agg_d2 = 0.0;
            agg_l2 = 0.0;
            for (int v = tid; v < V; v += g_threads) {
                const int r0 = vr0[v], c0 = coff[v], c1 = coff[v + 1];
                T acc = T(0) + (xn[r0] - ln[r0] * irho_n);
                double dsum = 0.0, lsum = 0.0;
                if (AGG) {
                    dsum = double(xn[r0]) - double(xc[r0]);
                    lsum = double(ln[r0]);
                }
                for (int q = c0 + 1; q < c1; ++q) {
                    const int r = crow[q];
                    acc += xn[r] - ln[r] * irho_n;
                    if (AGG) {
                        dsum += double(xn[r]) - double(xc[r]);
                        lsum += double(ln[r]);
                    }
                }
                ownp[v] = acc;
                publish(bnx, v, acc);
                if (AGG) {
                    dsum *= rho_c;
                    if (sbase[v] < 0) {
                        agg_d2 += dsum * dsum;
                        agg_l2 += lsum * lsum;
                    } else {
                        agg_publish(bp ^ 1, v, dsum, lsum);
                    }
                }
            }
            if (RHO) {
                rho_c = rho_n;
                rho_cT = in_vgpr(T(rho_n));
                irho_c = irho_n;
            }
            stamp(4);
            ++done;
            cur = nx;
            stamp(5);
        }
    }
    if (ok && !stopped) {
        // max_iter reached: the group sums of the last sweep, then the
        // sweeps not yet tested, in order
        result = done;
        if (AGG && done >= 1) {
            // the aggregated sums of the last sweep, which no further global
            // update completes
            if (wv != tw) {
                double ad2 = agg_d2, al2 = agg_l2;
                const int bp = int(done & 1);
                for (int v = tid; v < V; v += g_threads)
                    if (sbase[v] >= 0 && sme[v] == 0) agg_collect(bp, v, &ad2, &al2);
                agg_to_lds(ad2, al2);
            }
            __syncthreads();
            if (wv == tw && lane < 2) {
                double q = 0.0;
                for (int w = 0; w < n_work; ++w) q += aggw[w * 2 + lane];
                st_agent(ring1(done) + (5 + lane) * P + part, q);
            }
        }
        if (wv == tw && leader && done >= 1) {
            __builtin_amdgcn_s_waitcnt(0);
            issue_members(done);
            group_sums(done);
        }
        for (int64_t k = done > 3 ? done - 2 : 1; k <= done; ++k) {
            if (wv == tw) {
                issue_groups(k);
                totals(k, false);
            }
            __syncthreads();
            result = k;
            if (decide() || !ok) break;
            __syncthreads();  // tot is rewritten for the next sweep
        }
    }
    // ---- write the state of sweep `result` back (canonical order, FP64)
    const int fp = int(result % 3), fx = int(result & 3);
    for (int r = tid; r < R; r += nt) {
        const int canon = a.row_canon[pi.row_begin + r];
        a.xs[canon] = double(XS(fp)[r]);
        a.lam[canon] = double(LAM(fp)[r]);
    }
    if (result > 0)
        for (int v = tid; v < V; v += nt)
            if (a.var_writer[pi.var_begin + v]) a.x[a.var_gid[pi.var_begin + v]] = double(XL(fx)[v]);
    if (tid == 0 && (!ok || nonfinite)) atomicOr(&a.st->flags, (ok ? 0 : 1) | (nonfinite ? 2 : 0));
    if (part == 0 && tid == 0) {
        if (result > 0)
            for (int q = 0; q < nq; ++q) d[q] = tot[q];
        a.st->iters = result;
        a.st->computed = done;
        a.st->converged = converged;
        a.st->pres = sqrt(d[0]);
        a.st->dres = sqrt(AGG ? d[5] : d[1]);
        a.st->eps_p = sq * a.eps_abs + a.eps_rel * fmax(sqrt(d[2]), sqrt(d[3]));
        a.st->eps_d = sqd * a.eps_abs + a.eps_rel * sqrt(AGG ? d[6] : d[4]);
        a.st->rho = (RHO && result > 0) ? rho_of[result & 7] : a.rho;
    }
    if (RHO && part == 0 && wv == tw && lane == 0) {
        // the changes whose first sweep was reached (a change decided near
        // the end may fall after the returned sweep)
        int64_t nch = 0;
        const double* lg = rule_log;
        for (int64_t i = 0; i < rho_changes; ++i)
            if (int64_t(lg[2 * i]) <= result) ++nch;
        a.st->rho_changes = nch;
    }
    if (PROF && a.prof && tid == 0)
        for (int i = 0; i < 8; ++i)
            if (i != 6) a.prof[part * 8 + i] = double(tprof[i]);
    if (PROF && a.prof && wv == tw && lane == 0) a.prof[part * 8 + 6] = double(tw_prof);
}

template <typename T, int MODE>
__global__ __launch_bounds__(1024) void sweep_kernel(SweepArgs<T> a) {
    sweep_body<T, MODE>(a, blockIdx.x);
}

// Several independent problems in one launch: problem p's workgroups are the
// blocks first[p] .. first[p + 1] - 1, each running part blockIdx.x - first[p]
// of that problem's sweep. The problems share nothing but the launch: each
// has its own exchange words, residual rings, test and stop.
template <typename T, int MODE>
__global__ __launch_bounds__(1024) void sweep_many_kernel(const SweepArgs<T>* args, const int32_t* first, int32_t count) {
    int p = 0;
    while (p + 1 < count && int32_t(blockIdx.x) >= first[p + 1]) ++p;
    const SweepArgs<T> a = args[p];
    sweep_body<T, MODE>(a, unsigned(int32_t(blockIdx.x) - first[p]));
}

// Before every sweep launch, on the same stream: every exchange word empty,
// the status cleared (plain stores).
template <typename T>
__global__ void reset_sync_kernel(T* bpart, int64_t n_bwords, double* rpart, int64_t n_rwords, double* gpart,
                                  int64_t n_gwords, double* bagg, int64_t n_awords, SweepStatus* st) {
    const int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x, stride = int64_t(gridDim.x) * blockDim.x;
    using UB = typename Word<T>::U;
    using UR = typename Word<double>::U;
    for (int64_t i = i0; i < n_bwords; i += stride) reinterpret_cast<UB*>(bpart)[i] = Word<T>::kEmpty;
    for (int64_t i = i0; i < n_rwords; i += stride) reinterpret_cast<UR*>(rpart)[i] = Word<double>::kEmpty;
    for (int64_t i = i0; i < n_gwords; i += stride) reinterpret_cast<UR*>(gpart)[i] = Word<double>::kEmpty;
    for (int64_t i = i0; i < n_awords; i += stride) reinterpret_cast<UR*>(bagg)[i] = Word<double>::kEmpty;
    if (i0 == 0) {
        st->iters = 0;
        st->computed = 0;
        st->converged = 0;
        st->flags = 0;
        st->pres = st->dres = st->eps_p = st->eps_d = 0.0;
        st->rho = 0.0;
        st->rho_changes = 0;
    }
}

// ---------------------------------------------------------------------------
// Host launchers.

hipError_t launch_precompute(const PrecomputeArgs& a, hipStream_t stream) {
    const unsigned grid = unsigned((a.S + 3) / 4);
    if (a.max_n > 64 * 16) return hipErrorInvalidValue;
    if (a.max_n <= 64 * 4)
        hipLaunchKernelGGL(precompute_kernel<4>, dim3(grid), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(precompute_kernel<16>, dim3(grid), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T, int MODE>
static const void* sweep_ptr() {
    return reinterpret_cast<const void*>(&sweep_kernel<T, MODE>);
}

template <typename T, int MODE>
static const void* many_ptr() {
    return reinterpret_cast<const void*>(&sweep_many_kernel<T, MODE>);
}

template <typename T>
static const void* sweep_variant(int mode) {
    static const void* const table[8] = {sweep_ptr<T, 0>(), sweep_ptr<T, 1>(), sweep_ptr<T, 2>(), sweep_ptr<T, 3>(),
                                         sweep_ptr<T, 4>(), sweep_ptr<T, 5>(), sweep_ptr<T, 6>(), sweep_ptr<T, 7>()};
    return table[mode & 7];
}

template <typename T>
static const void* many_variant(int mode) {
    static const void* const table[8] = {many_ptr<T, 0>(), many_ptr<T, 1>(), many_ptr<T, 2>(), many_ptr<T, 3>(),
                                         many_ptr<T, 4>(), many_ptr<T, 5>(), many_ptr<T, 6>(), many_ptr<T, 7>()};
    return table[mode & 7];
}

template <typename T>
static int sweep_mode(const SweepArgs<T>& a) {
    return (a.prof ? kModeProf : 0) | (a.bagg ? kModeAgg : 0) | (a.rho_update ? kModeRho : 0);
}

hipError_t prepare_sweep(bool fp32, size_t lds_bytes) {
    for (int v = 0; v < 16; ++v) {
        const bool many = (v & 8) != 0;
        const void* f = fp32 ? (many ? many_variant<float>(v) : sweep_variant<float>(v))
                             : (many ? many_variant<double>(v) : sweep_variant<double>(v));
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t sweep_many_occupancy(bool fp32, int block, size_t lds_bytes, int* blocks_per_cu) {
    int best = 1 << 30;
    for (int v = 0; v < 8; ++v) {
        const void* f = fp32 ? many_variant<float>(v) : many_variant<double>(v);
        int n = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, lds_bytes);
        if (e != hipSuccess) return e;
        best = std::min(best, n);
    }
    *blocks_per_cu = best;
    return hipSuccess;
}

hipError_t sweep_occupancy(bool fp32, int block, size_t lds_bytes, int* blocks_per_cu) {
    // the fewest co-resident workgroups of any variant the handle may launch
    int best = 1 << 30;
    for (int v = 0; v < 8; ++v) {
        const void* f = fp32 ? sweep_variant<float>(v) : sweep_variant<double>(v);
        int n = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, lds_bytes);
        if (e != hipSuccess) return e;
        best = std::min(best, n);
    }
    *blocks_per_cu = best;
    return hipSuccess;
}

template <typename T>
static hipError_t reset_sync(const SweepArgs<T>& a, hipStream_t stream) {
    const int64_t nb = 2 * std::max<int64_t>(a.n_slots, 1), nr = int64_t(kRing) * a.P * 8;
    const int64_t ng = int64_t(kRing) * 8 * kGroup;
    const int64_t na = a.bagg ? 4 * std::max<int64_t>(a.n_slots, 1) : 0;
    const unsigned rgrid = unsigned(std::min<int64_t>(256, (std::max(std::max(nb, nr), na) + 255) / 256));
    hipLaunchKernelGGL(reset_sync_kernel<T>, dim3(rgrid), dim3(256), 0, stream, a.bpart, nb, a.rpart, nr, a.gpart, ng,
                       a.bagg, na, a.st);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_sweep_t(const SweepArgs<T>& a, int grid, int block, size_t lds, hipStream_t stream,
                                 bool cooperative) {
    hipError_t e = reset_sync(a, stream);
    if (e != hipSuccess) return e;
    SweepArgs<T> copy = a;
    void* args[] = {&copy};
    const void* f = sweep_variant<T>(sweep_mode(a));
    if (cooperative) return hipLaunchCooperativeKernel(f, dim3(grid), dim3(block), args, unsigned(lds), stream);
    return hipLaunchKernel(f, dim3(grid), dim3(block), args, lds, stream);
}

hipError_t launch_sweep(const SweepArgs<double>& a, int grid, int block, size_t lds, hipStream_t stream,
                        bool cooperative) {
    return launch_sweep_t<double>(a, grid, block, lds, stream, cooperative);
}
hipError_t launch_sweep(const SweepArgs<float>& a, int grid, int block, size_t lds, hipStream_t stream,
                        bool cooperative) {
    return launch_sweep_t<float>(a, grid, block, lds, stream, cooperative);
}

template <typename T>
static hipError_t launch_many_t(const std::vector<SweepArgs<T>>& host_args, const SweepArgs<T>* dev_args,
                                const int32_t* dev_first, int total_blocks, int block, size_t lds, hipStream_t stream) {
    for (const SweepArgs<T>& a : host_args) {
        const hipError_t e = reset_sync(a, stream);
        if (e != hipSuccess) return e;
    }
    int32_t count = int32_t(host_args.size());
    void* args[] = {const_cast<SweepArgs<T>**>(&dev_args), const_cast<int32_t**>(&dev_first), &count};
    // one variant for all: residual balancing if any problem asks for it (a
    // problem without it never changes rho there), the rest shared by all
    int mode = 0;
    for (const SweepArgs<T>& a : host_args) mode |= sweep_mode(a);
    const void* f = many_variant<T>(mode);
    return hipLaunchCooperativeKernel(f, dim3(total_blocks), dim3(block), args, unsigned(lds), stream);
}

hipError_t launch_sweep_many(const std::vector<SweepArgs<double>>& a, const SweepArgs<double>* dev_args,
                             const int32_t* dev_first, int total_blocks, int block, size_t lds, hipStream_t stream) {
    return launch_many_t<double>(a, dev_args, dev_first, total_blocks, block, lds, stream);
}
hipError_t launch_sweep_many(const std::vector<SweepArgs<float>>& a, const SweepArgs<float>* dev_args,
                             const int32_t* dev_first, int total_blocks, int block, size_t lds, hipStream_t stream) {
    return launch_many_t<float>(a, dev_args, dev_first, total_blocks, block, lds, stream);
}

}  // namespace ldopf
