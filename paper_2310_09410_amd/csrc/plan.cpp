// Work partition of the persistent sweep kernel (host-only).
//
// The subsystems are cut into P contiguous runs of a locality order (a
// depth-first walk of the feeder), one run per workgroup. Each workgroup
// keeps its run's operators and state in LDS for the whole solve. A global
// variable whose copies all sit in one run is interior: its clipped average
// (closed_1) is computed inside that workgroup. A variable shared by m runs
// is a boundary variable: every owner sends its partial sum of
// (x_k - lambda_k / rho) to each other owner through a slot of its own for
// that (writer, reader) pair, m^2 slots per variable with the reader's block
// of m first (slot base + reader * m + writer); each owner adds the m partial
// sums in owner order, so all owners compute the same value bit for bit.

#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"
#include "layout.h"

namespace ldopf {

namespace {

struct Cut {
    std::vector<int64_t> begin;  // P+1 boundaries into the order
};

Cut balanced_cut(const std::vector<double>& cost, int32_t P) {
    const int64_t S = int64_t(cost.size());
    std::vector<double> pre(S + 1, 0.0);
    for (int64_t i = 0; i < S; ++i) pre[i + 1] = pre[i] + cost[i];
    Cut c;
    c.begin.assign(P + 1, 0);
    c.begin[P] = S;
    int64_t pos = 0;
    for (int32_t p = 1; p < P; ++p) {
        const double target = pre[S] * double(p) / double(P);
        // first index whose prefix midpoint passes the target, keeping every
        // part non-empty
        int64_t i = std::max<int64_t>(pos + 1, 1);
        while (i < S - (P - p) && 0.5 * (pre[i] + pre[i + 1]) <= target) ++i;
        i = std::min<int64_t>(i, S - (P - p));
        c.begin[p] = i;
        pos = i;
    }
    return c;
}

}  // namespace

Plan make_plan(const ConsensusLP& lp, const std::vector<int32_t>& rank, bool fp32,
               int32_t rows_per_part, int32_t block_threads, int32_t max_parts,
               int64_t max_lds_bytes) {
    const int64_t S = lp.S;
    const uint32_t w = fp32 ? 4u : 8u;
    std::vector<int64_t> order = lp.locality_order;
    if (order.empty()) {
        order.resize(S);
        std::iota(order.begin(), order.end(), 0);
    }
    std::vector<int32_t> K(S), mode(S);
    std::vector<int64_t> boff(S + 1, 0);
    int64_t rank_words = 0;
    for (int64_t s = 0; s < S; ++s) {
        const int32_t n = lp.ns[s], r = rank[s];
        if (n > kMaxSubsystemVars)
            fail(LDOPF_UNSUPPORTED, "subsystem " + std::to_string(s) + " has more than " + std::to_string(kMaxSubsystemVars) +
                                        " variables");
        // rank form: the row-space basis if it is the smaller side, else the
        // basis of its orthogonal complement
        mode[s] = (r <= n - r) ? 1 : 0;
        K[s] = std::min(r, n - r);
        boff[s + 1] = boff[s] + int64_t(n) * n;
        rank_words += int64_t(n) * K[s];
    }
    std::vector<double> cost(S);
    for (int64_t i = 0; i < S; ++i) {
        const int64_t s = order[i];
        const int32_t n = lp.ns[s];
        cost[i] = double(w) * (double(n) * K[s] + 7.0 * n + K[s] + 6.0 * n) + 6.0 * n + 2.0 * K[s] + 16.0;
    }
    const int64_t nloc = lp.loc_off[S];
    const int32_t rpp = rows_per_part > 0 ? rows_per_part : 512;
    int32_t cap = int32_t(std::min<int64_t>(max_parts, S));
    if (cap < 1) cap = 1;
    int32_t P = int32_t(std::min<int64_t>(cap, std::max<int64_t>(1, (nloc + rpp - 1) / rpp)));
    const uint32_t waves_budget = 16;

    std::vector<int32_t> stamp(lp.n, -1), lidx(lp.n, 0);
    while (true) {
        Cut cut = balanced_cut(cost, P);
        Plan pl;
        pl.n_parts = P;
        pl.rank_words = rank_words;
        pl.parts.resize(P);
        std::fill(stamp.begin(), stamp.end(), -1);
        std::vector<int32_t> owner_count(lp.n, 0);
        int64_t max_rows = 0, max_lds = 0;
        bool fits = true;
        for (int32_t p = 0; p < P; ++p) {
            PartInfo& pi = pl.parts[p];
            pi.sub_begin = int32_t(pl.subs.size());
            pi.row_begin = int32_t(pl.row_canon.size());
            pi.var_begin = int32_t(pl.var_gid.size());
            pi.tk_begin = int32_t(pl.tk_sub.size());
            pi.copy_begin = int32_t(pl.var_copy_rows.size());
            pi.coff_begin = int32_t(pl.var_copy_off.size());
            uint32_t row = 0, t = 0, wwords = 0, nv = 0;
            for (int64_t i = cut.begin[p]; i < cut.begin[p + 1]; ++i) {
                const int64_t s = order[i];
                const int32_t n = lp.ns[s];
                SubMeta m{};
                m.row0 = uint16_t(row);
                m.n = uint16_t(n);
                m.k = uint16_t(K[s]);
                m.t0 = uint16_t(t);
                m.mode = uint16_t(mode[s]);
                m.w0 = wwords;
                m.canon = uint32_t(s);
                m.basis = uint64_t(boff[s]);
                m.brow = uint32_t(mode[s] ? 0 : rank[s]);
                const uint16_t local_sub = uint16_t(pl.subs.size() - pi.sub_begin);
                pl.subs.push_back(m);
                for (int32_t k = 0; k < K[s]; ++k) pl.tk_sub.push_back(local_sub);
                for (int32_t j = 0; j < n; ++j) {
                    const int64_t canon = lp.loc_off[s] + j;
                    const int64_t g = lp.gidx[canon];
                    if (stamp[g] != p) {
                        stamp[g] = p;
                        lidx[g] = int32_t(nv++);
                        pl.var_gid.push_back(int32_t(g));
                        owner_count[g]++;
                    }
                    pl.row_canon.push_back(int32_t(canon));
                    pl.row_lvar.push_back(uint16_t(lidx[g] & 0xffff));
                    pl.row_sub.push_back(local_sub);
                }
                row += uint32_t(n);
                t += uint32_t(K[s]);
                wwords += uint32_t(n) * uint32_t(K[s]);
            }
            pi.n_sub = int32_t(pl.subs.size()) - pi.sub_begin;
            pi.n_row = int32_t(row);
            pi.n_var = int32_t(nv);
            pi.n_tk = int32_t(t);
            pi.w_words = int32_t(wwords);
            // the kernel packs operator offsets, rows and tasks in 16 bits
            if (row > 65535 || nv > 65535 || t > 65535 || wwords > 65535) fits = false;
            // copies of each part-local var, in row order
            std::vector<uint16_t> cnt(nv + 1, 0);
            for (uint32_t r = 0; r < row; ++r) cnt[pl.row_lvar[pi.row_begin + r] + 1]++;
            for (uint32_t v = 0; v < nv; ++v) cnt[v + 1] = uint16_t(cnt[v + 1] + cnt[v]);
            std::vector<uint16_t> fillpos(cnt.begin(), cnt.end() - 1);
            std::vector<uint16_t> rows_of(row);
            for (uint32_t r = 0; r < row; ++r) rows_of[fillpos[pl.row_lvar[pi.row_begin + r]]++] = uint16_t(r);
            pl.var_copy_off.insert(pl.var_copy_off.end(), cnt.begin(), cnt.end());
            pl.var_copy_rows.insert(pl.var_copy_rows.end(), rows_of.begin(), rows_of.end());
            const LdsLayout L = lds_layout(w, wwords, row, t, nv, uint32_t(pi.n_sub), waves_budget);
            pi.lds_bytes = int32_t(L.total);
            max_rows = std::max<int64_t>(max_rows, row);
            max_lds = std::max<int64_t>(max_lds, L.total);
            if (int64_t(L.total) > max_lds_bytes) fits = false;
        }
        if (!fits) {
            if (P >= cap) {
                fail(LDOPF_UNSUPPORTED, "problem too large for the LDS-resident sweep: " + std::to_string(max_lds) +
                                            " bytes per workgroup with " + std::to_string(P) + " workgroups");
            }
            P = std::min<int32_t>(cap, std::max<int32_t>(P + 1, int32_t(std::ceil(P * 1.15))));
            continue;
        }
        // boundary slots: owner_count^2 per shared variable, owners in part order
        std::vector<int32_t> slot_lo(lp.n, -1), seen(lp.n, 0);
        int64_t slots = 0;
        for (int64_t g = 0; g < lp.n; ++g)
            if (owner_count[g] > 1) {
                slot_lo[g] = int32_t(slots);
                slots += int64_t(owner_count[g]) * owner_count[g];
                if (slots >= (int64_t(1) << 30)) fail(LDOPF_UNSUPPORTED, "too many boundary slots");
            }
        pl.n_slots = int32_t(slots);
        const size_t nvar_total = pl.var_gid.size();
        pl.var_slot.assign(nvar_total, -1);
        pl.var_slot_lo.assign(nvar_total, -1);
        pl.var_slot_hi.assign(nvar_total, -1);
        pl.var_writer.assign(nvar_total, 0);
        for (int32_t p = 0; p < P; ++p) {
            const PartInfo& pi = pl.parts[p];
            for (int32_t v = 0; v < pi.n_var; ++v) {
                const size_t q = size_t(pi.var_begin) + v;
                const int32_t g = pl.var_gid[q];
                const int32_t my = seen[g]++;
                pl.var_writer[q] = my == 0;
                if (owner_count[g] > 1) {
                    pl.var_slot[q] = my;                // this part's owner index
                    pl.var_slot_lo[q] = slot_lo[g];     // slot base
                    pl.var_slot_hi[q] = owner_count[g]; // owners m
                }
            }
        }
        int32_t bt = block_threads;
        // one row per lane of the work waves, plus the wave that runs the
        // termination test
        if (bt <= 0) bt = int32_t(std::min<int64_t>(1024, std::max<int64_t>(1, (max_rows + 63) / 64) * 64 + 64));
        if (bt < 128 || bt > 1024 || bt % 64 != 0) fail(LDOPF_INVALID_ARGUMENT, "block_threads must be a multiple of 64 in [128, 1024]");
        pl.block_threads = bt;
        // recompute the LDS need with the real wave count
        int64_t lds = 0;
        for (auto& pi : pl.parts) {
            const LdsLayout L = lds_layout(w, uint32_t(pi.w_words), uint32_t(pi.n_row), uint32_t(pi.n_tk),
                                           uint32_t(pi.n_var), uint32_t(pi.n_sub), uint32_t(bt / 64));
            pi.lds_bytes = int32_t(L.total);
            lds = std::max<int64_t>(lds, L.total);
        }
        pl.lds_bytes = lds;
        return pl;
    }
}

}  // namespace ldopf
