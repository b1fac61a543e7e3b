// Network -> consensus LP: the rows of Section II-A (power balance, the
// voltage-dependent load model, the linearized power flow), the global
// variable order of LP_model, and the decomposition of Section V-A (one
// subsystem per line and per bus, leaf buses merged into their line).
//
// Host-only code; no HIP calls. The subsystem variable sets are structural:
// a subsystem holds every variable its component's equations name, even where
// a coefficient happens to be zero, so the number of copies of a variable
// (and with it the consensus averaging) never depends on data values.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>

#include "internal.h"

namespace ldopf {

namespace {

constexpr double kSqrt3 = 1.7320508075688772935;

inline bool has_phase(unsigned mask, int ph) { return (mask >> ph) & 1u; }
// Position of phase ph among the phases of mask (a, b, c ascending).
inline int phase_slot(unsigned mask, int ph) { return __builtin_popcount(mask & ((1u << ph) - 1u)); }

// Read-only view of the network with the documented defaults for nullable arrays.
struct View {
    const ldopf_network& n;
    static double at(const double* p, int64_t i, int ph, double dflt) { return p ? p[i * 3 + ph] : dflt; }
    double wlo(int64_t i, int ph) const { return at(n.bus_wlo, i, ph, -INFINITY); }
    double whi(int64_t i, int ph) const { return at(n.bus_whi, i, ph, INFINITY); }
    double gsh(int64_t i, int ph) const { return at(n.bus_gsh, i, ph, 0.0); }
    double bsh(int64_t i, int ph) const { return at(n.bus_bsh, i, ph, 0.0); }
    double gs_i(int64_t e, int ph) const { return at(n.line_gs_from, e, ph, 0.0); }
    double bs_i(int64_t e, int ph) const { return at(n.line_bs_from, e, ph, 0.0); }
    double gs_j(int64_t e, int ph) const { return at(n.line_gs_to, e, ph, 0.0); }
    double bs_j(int64_t e, int ph) const { return at(n.line_bs_to, e, ph, 0.0); }
    double tau(int64_t e, int ph) const { return at(n.line_tau, e, ph, 1.0); }
    double alpha(int64_t l, int ph) const { return at(n.load_alpha, l, ph, 0.0); }
    double beta(int64_t l, int ph) const { return at(n.load_beta, l, ph, 0.0); }
    int conn(int64_t l) const { return n.load_conn ? n.load_conn[l] : 0; }
};

// Global index of every variable (block order of LP_model).
struct Layout {
    std::vector<int64_t> gen0, bus0, load0, line0;
    std::vector<uint8_t> is_voltage;
    int64_t n = 0;
    const ldopf_network* net = nullptr;
    int64_t pg(int k, int ph) const { return gen0[k] + 2 * phase_slot(net->gen_phases[k], ph); }
    int64_t qg(int k, int ph) const { return pg(k, ph) + 1; }
    int64_t w(int i, int ph) const { return bus0[i] + phase_slot(net->bus_phases[i], ph); }
    int64_t load(int l, int ph, int which) const { return load0[l] + 4 * phase_slot(net->load_phases[l], ph) + which; }
    int64_t flow(int e, int ph, int which) const { return line0[e] + 4 * phase_slot(net->line_phases[e], ph) + which; }
};
enum { PB = 0, QB = 1, PD = 2, QD = 3 };
enum { PIJ = 0, QIJ = 1, PJI = 2, QJI = 3 };

Layout make_layout(const ldopf_network& net) {
    Layout L;
    L.net = &net;
    int64_t pos = 0;
    L.gen0.resize(net.n_gen);
    for (int k = 0; k < net.n_gen; ++k) { L.gen0[k] = pos; pos += 2 * __builtin_popcount(net.gen_phases[k]); }
    L.bus0.resize(net.n_bus);
    int64_t wbeg = pos;
    for (int i = 0; i < net.n_bus; ++i) { L.bus0[i] = pos; pos += __builtin_popcount(net.bus_phases[i]); }
    int64_t wend = pos;
    L.load0.resize(net.n_load);
    for (int l = 0; l < net.n_load; ++l) { L.load0[l] = pos; pos += 4 * __builtin_popcount(net.load_phases[l]); }
    L.line0.resize(net.n_line);
    for (int e = 0; e < net.n_line; ++e) { L.line0[e] = pos; pos += 4 * __builtin_popcount(net.line_phases[e]); }
    L.n = pos;
    L.is_voltage.assign(pos, 0);
    for (int64_t v = wbeg; v < wend; ++v) L.is_voltage[v] = 1;
    return L;
}

bool finite_or_null(const double* p, int64_t count) {
    if (!p) return true;
    for (int64_t t = 0; t < count; ++t)
        if (std::isnan(p[t])) return false;
    return true;
}

void validate(const ldopf_network& net) {
    if (net.n_bus < 1 || net.n_line < 0 || net.n_load < 0 || net.n_gen < 0)
        fail(LDOPF_INVALID_ARGUMENT, "network counts must be n_bus >= 1 and the others >= 0");
    if (net.root < 0 || net.root >= net.n_bus) fail(LDOPF_INVALID_NETWORK, "root bus out of range");
    if (!net.bus_phases) fail(LDOPF_INVALID_ARGUMENT, "bus_phases is required");
    if (net.n_line > 0 && (!net.line_from || !net.line_to || !net.line_phases || !net.line_r || !net.line_x))
        fail(LDOPF_INVALID_ARGUMENT, "line_from, line_to, line_phases, line_r, line_x are required");
    if (net.n_load > 0 && (!net.load_bus || !net.load_phases || !net.load_a || !net.load_b))
        fail(LDOPF_INVALID_ARGUMENT, "load_bus, load_phases, load_a, load_b are required");
    if (net.n_gen > 0 && (!net.gen_bus || !net.gen_phases))
        fail(LDOPF_INVALID_ARGUMENT, "gen_bus and gen_phases are required");
    auto bad_mask = [](unsigned m) { return m == 0 || m > 7; };
    for (int i = 0; i < net.n_bus; ++i)
        if (bad_mask(net.bus_phases[i])) fail(LDOPF_INVALID_NETWORK, "bus " + std::to_string(i) + ": phase set must be a nonempty subset of abc");
    for (int e = 0; e < net.n_line; ++e) {
        int i = net.line_from[e], j = net.line_to[e];
        if (i < 0 || i >= net.n_bus || j < 0 || j >= net.n_bus || i == j)
            fail(LDOPF_INVALID_NETWORK, "line " + std::to_string(e) + ": end buses out of range or equal");
        unsigned m = net.line_phases[e];
        if (bad_mask(m) || (m & ~net.bus_phases[i]) || (m & ~net.bus_phases[j]))
            fail(LDOPF_INVALID_NETWORK, "line " + std::to_string(e) + ": phase set must be a subset of both end buses' phases");
    }
    for (int l = 0; l < net.n_load; ++l) {
        int i = net.load_bus[l];
        if (i < 0 || i >= net.n_bus) fail(LDOPF_INVALID_NETWORK, "load " + std::to_string(l) + ": bus out of range");
        unsigned m = net.load_phases[l];
        if (bad_mask(m) || (m & ~net.bus_phases[i]))
            fail(LDOPF_INVALID_NETWORK, "load " + std::to_string(l) + ": phase set must be a subset of its bus's phases");
        int conn = net.load_conn ? net.load_conn[l] : 0;
        if (conn != 0 && conn != 1) fail(LDOPF_INVALID_NETWORK, "load " + std::to_string(l) + ": connection must be 0 (wye) or 1 (delta)");
        if (conn == 1 && m != 7) fail(LDOPF_INVALID_NETWORK, "load " + std::to_string(l) + ": a delta load must be three-phase");
    }
    for (int k = 0; k < net.n_gen; ++k) {
        int i = net.gen_bus[k];
        if (i < 0 || i >= net.n_bus) fail(LDOPF_INVALID_NETWORK, "generator " + std::to_string(k) + ": bus out of range");
        unsigned m = net.gen_phases[k];
        if (bad_mask(m) || (m & ~net.bus_phases[i]))
            fail(LDOPF_INVALID_NETWORK, "generator " + std::to_string(k) + ": phase set must be a subset of its bus's phases");
    }
    const int64_t B3 = int64_t(net.n_bus) * 3, E3 = int64_t(net.n_line) * 3, D3 = int64_t(net.n_load) * 3,
                  G3 = int64_t(net.n_gen) * 3;
    bool ok = finite_or_null(net.bus_wlo, B3) && finite_or_null(net.bus_whi, B3) && finite_or_null(net.bus_gsh, B3) &&
              finite_or_null(net.bus_bsh, B3) && finite_or_null(net.line_r, E3 * 3) && finite_or_null(net.line_x, E3 * 3) &&
              finite_or_null(net.line_gs_from, E3) && finite_or_null(net.line_bs_from, E3) &&
              finite_or_null(net.line_gs_to, E3) && finite_or_null(net.line_bs_to, E3) && finite_or_null(net.line_tau, E3) &&
              finite_or_null(net.line_plo, E3) && finite_or_null(net.line_phi, E3) && finite_or_null(net.line_qlo, E3) &&
              finite_or_null(net.line_qhi, E3) && finite_or_null(net.load_a, D3) && finite_or_null(net.load_b, D3) &&
              finite_or_null(net.load_alpha, D3) && finite_or_null(net.load_beta, D3) && finite_or_null(net.gen_plo, G3) &&
              finite_or_null(net.gen_phi, G3) && finite_or_null(net.gen_qlo, G3) && finite_or_null(net.gen_qhi, G3) &&
              finite_or_null(net.gen_cost_p, G3) && finite_or_null(net.gen_cost_q, G3);
    if (!ok) fail(LDOPF_INVALID_NETWORK, "NaN in network data");
    auto inf_ok = [](const double* p, int64_t count) {
        if (!p) return true;
        for (int64_t t = 0; t < count; ++t)
            if (std::isinf(p[t])) return false;
        return true;
    };
    if (!inf_ok(net.line_r, E3 * 3) || !inf_ok(net.line_x, E3 * 3) || !inf_ok(net.load_a, D3) || !inf_ok(net.load_b, D3) ||
        !inf_ok(net.load_alpha, D3) || !inf_ok(net.load_beta, D3) || !inf_ok(net.bus_gsh, B3) || !inf_ok(net.bus_bsh, B3) ||
        !inf_ok(net.line_tau, E3) || !inf_ok(net.gen_cost_p, G3) || !inf_ok(net.gen_cost_q, G3) ||
        !inf_ok(net.line_gs_from, E3) || !inf_ok(net.line_bs_from, E3) || !inf_ok(net.line_gs_to, E3) ||
        !inf_ok(net.line_bs_to, E3))
        fail(LDOPF_INVALID_NETWORK, "infinite coefficient in network data");
}

// M^p and M^q entry (phi, psi) of a line: -2r, -2x on the diagonal; for the
// phase that follows phi in the cycle a -> b -> c -> a the pair
// (r - sqrt3 x, x + sqrt3 r), for the phase that precedes it (r + sqrt3 x,
// x - sqrt3 r).
void m_entry(const double* r9, const double* x9, int phi, int psi, double& mp, double& mq) {
    const double r = r9[phi * 3 + psi], x = x9[phi * 3 + psi];
    if (phi == psi) {
        mp = -2.0 * r;
        mq = -2.0 * x;
    } else if (psi == (phi + 1) % 3) {
        mp = r - kSqrt3 * x;
        mq = x + kSqrt3 * r;
    } else {
        mp = r + kSqrt3 * x;
        mq = x - kSqrt3 * r;
    }
}

struct Row {
    std::vector<std::pair<int64_t, double>> a;
    double rhs = 0.0;
    int32_t load = -1;    // load whose reference power this row carries
    int64_t wglob = -1;   // global index of the load-scaled w coefficient
    void add(int64_t col, double v) { a.emplace_back(col, v); }
};

struct Builder {
    const ldopf_network& net;
    const View V;
    const Layout& L;
    const std::vector<std::vector<int32_t>>& lines_at;
    const std::vector<std::vector<int32_t>>& loads_at;
    const std::vector<std::vector<int32_t>>& gens_at;
    std::vector<Row> rows;
    std::vector<int64_t> vars;

    void line_part(int e) {
        const int i = net.line_from[e], j = net.line_to[e];
        const unsigned m = net.line_phases[e];
        const double* r9 = net.line_r + int64_t(e) * 9;
        const double* x9 = net.line_x + int64_t(e) * 9;
        for (int f = 0; f < 3; ++f) {
            if (!has_phase(m, f)) continue;
            Row loss_p, loss_q, drop;
            // p_ij + p_ji = gs_i w_i + gs_j w_j
            loss_p.add(L.flow(e, f, PIJ), 1.0);
            loss_p.add(L.flow(e, f, PJI), 1.0);
            loss_p.add(L.w(i, f), -V.gs_i(e, f));
            loss_p.add(L.w(j, f), -V.gs_j(e, f));
            // q_ij + q_ji = -bs_i w_i - bs_j w_j
            loss_q.add(L.flow(e, f, QIJ), 1.0);
            loss_q.add(L.flow(e, f, QJI), 1.0);
            loss_q.add(L.w(i, f), V.bs_i(e, f));
            loss_q.add(L.w(j, f), V.bs_j(e, f));
            // w_i = tau w_j - sum_psi Mp (p_ij - gs w_i) - sum_psi Mq (q_ij + bs w_i)
            drop.add(L.w(i, f), 1.0);
            drop.add(L.w(j, f), -V.tau(e, f));
            for (int g = 0; g < 3; ++g) {
                if (!has_phase(m, g)) continue;
                double mp, mq;
                m_entry(r9, x9, f, g, mp, mq);
                drop.add(L.flow(e, g, PIJ), mp);
                drop.add(L.flow(e, g, QIJ), mq);
                drop.add(L.w(i, g), -mp * V.gs_i(e, g) + mq * V.bs_i(e, g));
            }
            rows.push_back(std::move(loss_p));
            rows.push_back(std::move(loss_q));
            rows.push_back(std::move(drop));
            for (int which = 0; which < 4; ++which) vars.push_back(L.flow(e, f, which));
            vars.push_back(L.w(i, f));
            vars.push_back(L.w(j, f));
        }
    }

    void load_part(int l) {
        const int i = net.load_bus[l];
        const unsigned m = net.load_phases[l];
        const double* a = net.load_a + int64_t(l) * 3;
        const double* b = net.load_b + int64_t(l) * 3;
        for (int f = 0; f < 3; ++f)
            if (has_phase(m, f))
                for (int which = 0; which < 4; ++which) vars.push_back(L.load(l, f, which));
        if (V.conn(l) == 0) {
            for (int f = 0; f < 3; ++f) {
                if (!has_phase(m, f)) continue;
                const double al = V.alpha(l, f), be = V.beta(l, f);
                Row rp, rq, ep, eq;
                rp.add(L.load(l, f, PD), 1.0);
                rp.add(L.w(i, f), -0.5 * a[f] * al);
                rp.rhs = a[f] - 0.5 * a[f] * al;
                rp.load = l;
                rp.wglob = L.w(i, f);
                rq.add(L.load(l, f, QD), 1.0);
                rq.add(L.w(i, f), -0.5 * b[f] * be);
                rq.rhs = b[f] - 0.5 * b[f] * be;
                rq.load = l;
                rq.wglob = L.w(i, f);
                ep.add(L.load(l, f, PB), 1.0);
                ep.add(L.load(l, f, PD), -1.0);
                eq.add(L.load(l, f, QB), 1.0);
                eq.add(L.load(l, f, QD), -1.0);
                rows.push_back(std::move(rp));
                rows.push_back(std::move(rq));
                rows.push_back(std::move(ep));
                rows.push_back(std::move(eq));
            }
            return;
        }
        // delta: w-hat = 3 w in the two model rows of each phase
        for (int f = 0; f < 3; ++f) {
            Row r;
            r.add(L.load(l, f, PD), 1.0);
            r.add(L.w(i, f), -1.5 * a[f] * V.alpha(l, f));
            r.rhs = a[f] - 0.5 * a[f] * V.alpha(l, f);
            r.load = l;
            r.wglob = L.w(i, f);
            rows.push_back(std::move(r));
        }
        for (int f = 0; f < 3; ++f) {
            Row r;
            r.add(L.load(l, f, QD), 1.0);
            r.add(L.w(i, f), -1.5 * b[f] * V.beta(l, f));
            r.rhs = b[f] - 0.5 * b[f] * V.beta(l, f);
            r.load = l;
            r.wglob = L.w(i, f);
            rows.push_back(std::move(r));
        }
        Row sp, sq;
        for (int f = 0; f < 3; ++f) {
            sp.add(L.load(l, f, PB), 1.0);
            sp.add(L.load(l, f, PD), -1.0);
            sq.add(L.load(l, f, QB), 1.0);
            sq.add(L.load(l, f, QD), -1.0);
        }
        rows.push_back(std::move(sp));
        rows.push_back(std::move(sq));
        auto pb = [&](int f) { return L.load(l, f, PB); };
        auto qb = [&](int f) { return L.load(l, f, QB); };
        auto pd = [&](int f) { return L.load(l, f, PD); };
        auto qd = [&](int f) { return L.load(l, f, QD); };
        const double h = 0.5, s = 0.5 * kSqrt3;
        Row c1, c2, c3, c4;  // coupling rows, phases a, b, c = 0, 1, 2
        c1.add(pb(1), 1.5); c1.add(qb(1), -s); c1.add(pd(1), -1.0); c1.add(pd(0), -h); c1.add(qd(0), s);
        c2.add(pb(1), s); c2.add(qb(1), 1.5); c2.add(pd(0), -s); c2.add(qd(0), -h); c2.add(qd(1), -1.0);
        c3.add(qb(1), kSqrt3); c3.add(pb(2), 1.5); c3.add(qb(2), -s); c3.add(pd(0), -h); c3.add(qd(0), -s); c3.add(pd(2), -1.0);
        c4.add(pb(1), -kSqrt3); c4.add(pb(2), s); c4.add(qb(2), 1.5); c4.add(pd(0), s); c4.add(qd(0), -h); c4.add(qd(2), -1.0);
        rows.push_back(std::move(c1));
        rows.push_back(std::move(c2));
        rows.push_back(std::move(c3));
        rows.push_back(std::move(c4));
    }

    void bus_part(int i) {
        const unsigned m = net.bus_phases[i];
        for (int f = 0; f < 3; ++f) {
            if (!has_phase(m, f)) continue;
            Row rp, rq;
            for (int e : lines_at[i]) {
                if (!has_phase(net.line_phases[e], f)) continue;
                const bool from = net.line_from[e] == i;
                rp.add(L.flow(e, f, from ? PIJ : PJI), 1.0);
                rq.add(L.flow(e, f, from ? QIJ : QJI), 1.0);
            }
            for (int l : loads_at[i]) {
                if (!has_phase(net.load_phases[l], f)) continue;
                rp.add(L.load(l, f, PB), 1.0);
                rq.add(L.load(l, f, QB), 1.0);
            }
            rp.add(L.w(i, f), V.gsh(i, f));
            rq.add(L.w(i, f), -V.bsh(i, f));
            for (int k : gens_at[i]) {
                if (!has_phase(net.gen_phases[k], f)) continue;
                rp.add(L.pg(k, f), -1.0);
                rq.add(L.qg(k, f), -1.0);
            }
            rows.push_back(std::move(rp));
            rows.push_back(std::move(rq));
            vars.push_back(L.w(i, f));
        }
        for (int e : lines_at[i]) {
            const bool from = net.line_from[e] == i;
            for (int f = 0; f < 3; ++f) {
                if (!has_phase(net.line_phases[e], f)) continue;
                vars.push_back(L.flow(e, f, from ? PIJ : PJI));
                vars.push_back(L.flow(e, f, from ? QIJ : QJI));
            }
        }
        for (int k : gens_at[i])
            for (int f = 0; f < 3; ++f)
                if (has_phase(net.gen_phases[k], f)) {
                    vars.push_back(L.pg(k, f));
                    vars.push_back(L.qg(k, f));
                }
        for (int l : loads_at[i]) load_part(l);
    }

    // Dense A_s over the sorted structural variable set; appended to lp.
    void emit(ConsensusLP& lp) {
        std::sort(vars.begin(), vars.end());
        vars.erase(std::unique(vars.begin(), vars.end()), vars.end());
        const int64_t n = int64_t(vars.size()), m = int64_t(rows.size());
        const int64_t a0 = int64_t(lp.A.size());
        lp.A.resize(a0 + m * n, 0.0);
        for (int64_t r = 0; r < m; ++r) {
            for (auto& [col, v] : rows[r].a) {
                auto it = std::lower_bound(vars.begin(), vars.end(), col);
                lp.A[a0 + r * n + (it - vars.begin())] += v;
            }
            lp.b.push_back(rows[r].rhs);
            lp.row_load.push_back(rows[r].load);
            int32_t wc = -1;
            if (rows[r].wglob >= 0)
                wc = int32_t(std::lower_bound(vars.begin(), vars.end(), rows[r].wglob) - vars.begin());
            lp.row_wcol.push_back(wc);
        }
        lp.gidx.insert(lp.gidx.end(), vars.begin(), vars.end());
        lp.ns.push_back(int32_t(n));
        lp.ms.push_back(int32_t(m));
        rows.clear();
        vars.clear();
    }
};

}  // namespace

ConsensusLP assemble_network(const ldopf_network& net) {
    validate(net);
    const View V{net};
    Layout L = make_layout(net);
    ConsensusLP lp;
    lp.n = L.n;
    lp.n_load = net.n_load;
    lp.c.assign(L.n, 0.0);
    lp.lo.assign(L.n, -INFINITY);
    lp.hi.assign(L.n, INFINITY);
    for (int k = 0; k < net.n_gen; ++k)
        for (int f = 0; f < 3; ++f) {
            if (!has_phase(net.gen_phases[k], f)) continue;
            lp.lo[L.pg(k, f)] = View::at(net.gen_plo, k, f, -INFINITY);
            lp.hi[L.pg(k, f)] = View::at(net.gen_phi, k, f, INFINITY);
            lp.lo[L.qg(k, f)] = View::at(net.gen_qlo, k, f, -INFINITY);
            lp.hi[L.qg(k, f)] = View::at(net.gen_qhi, k, f, INFINITY);
            lp.c[L.pg(k, f)] = View::at(net.gen_cost_p, k, f, 1.0);
            lp.c[L.qg(k, f)] = View::at(net.gen_cost_q, k, f, 0.0);
        }
    for (int i = 0; i < net.n_bus; ++i)
        for (int f = 0; f < 3; ++f)
            if (has_phase(net.bus_phases[i], f)) {
                lp.lo[L.w(i, f)] = V.wlo(i, f);
                lp.hi[L.w(i, f)] = V.whi(i, f);
            }
    for (int e = 0; e < net.n_line; ++e)
        for (int f = 0; f < 3; ++f) {
            if (!has_phase(net.line_phases[e], f)) continue;
            const double plo = View::at(net.line_plo, e, f, -INFINITY), phi = View::at(net.line_phi, e, f, INFINITY);
            const double qlo = View::at(net.line_qlo, e, f, -INFINITY), qhi = View::at(net.line_qhi, e, f, INFINITY);
            lp.lo[L.flow(e, f, PIJ)] = plo; lp.hi[L.flow(e, f, PIJ)] = phi;
            lp.lo[L.flow(e, f, PJI)] = plo; lp.hi[L.flow(e, f, PJI)] = phi;
            lp.lo[L.flow(e, f, QIJ)] = qlo; lp.hi[L.flow(e, f, QIJ)] = qhi;
            lp.lo[L.flow(e, f, QJI)] = qlo; lp.hi[L.flow(e, f, QJI)] = qhi;
        }
    for (int64_t v = 0; v < L.n; ++v)
        if (lp.lo[v] > lp.hi[v]) fail(LDOPF_INFEASIBLE_BOUNDS, "global variable " + std::to_string(v) + ": lower bound above upper bound");
    // Starting value of the copies (Section V-A): 1 for a squared voltage,
    // the midpoint of two finite bounds, else 0 clipped into the box.
    lp.x_init.resize(L.n);
    for (int64_t v = 0; v < L.n; ++v) {
        double s = std::min(std::max(0.0, lp.lo[v]), lp.hi[v]);
        if (std::isfinite(lp.lo[v]) && std::isfinite(lp.hi[v])) s = 0.5 * (lp.lo[v] + lp.hi[v]);
        if (L.is_voltage[v]) s = 1.0;
        lp.x_init[v] = s;
    }

    std::vector<std::vector<int32_t>> lines_at(net.n_bus), loads_at(net.n_bus), gens_at(net.n_bus);
    for (int e = 0; e < net.n_line; ++e) {
        lines_at[net.line_from[e]].push_back(e);
        lines_at[net.line_to[e]].push_back(e);
    }
    for (int l = 0; l < net.n_load; ++l) loads_at[net.load_bus[l]].push_back(l);
    for (int k = 0; k < net.n_gen; ++k) gens_at[net.gen_bus[k]].push_back(k);
    std::vector<uint8_t> leaf(net.n_bus, 0);
    for (int i = 0; i < net.n_bus; ++i) leaf[i] = (i != net.root && lines_at[i].size() == 1);

    Builder B{net, V, L, lines_at, loads_at, gens_at, {}, {}};
    for (int e = 0; e < net.n_line; ++e) {
        B.line_part(e);
        for (int end : {net.line_from[e], net.line_to[e]})
            if (leaf[end]) B.bus_part(end);
        B.emit(lp);
    }
    std::vector<int64_t> bus_sub(net.n_bus, -1);
    int64_t s = net.n_line;
    for (int i = 0; i < net.n_bus; ++i) {
        if (leaf[i]) continue;
        B.bus_part(i);
        B.emit(lp);
        bus_sub[i] = s++;
    }
    lp.S = s;

    // Depth-first walk from the root: a bus subsystem, then each incident
    // line's subsystem followed by the subtree behind it.
    std::vector<uint8_t> bus_seen(net.n_bus, 0), line_seen(net.n_line, 0);
    std::vector<std::pair<int32_t, size_t>> stack;
    auto visit_bus = [&](int32_t i) {
        bus_seen[i] = 1;
        if (bus_sub[i] >= 0) lp.locality_order.push_back(bus_sub[i]);
        stack.emplace_back(i, 0);
    };
    for (int32_t start0 = -1; start0 < net.n_bus; ++start0) {
        const int32_t start = start0 < 0 ? net.root : start0;
        if (bus_seen[start]) continue;
        visit_bus(start);
        while (!stack.empty()) {
            const int32_t b = stack.back().first;
            const size_t p = stack.back().second;
            if (p >= lines_at[b].size()) {
                stack.pop_back();
                continue;
            }
            stack.back().second = p + 1;
            const int32_t e = lines_at[b][p];
            if (line_seen[e]) continue;
            line_seen[e] = 1;
            lp.locality_order.push_back(e);
            const int32_t j = net.line_from[e] == b ? net.line_to[e] : net.line_from[e];
            if (!bus_seen[j]) visit_bus(j);
        }
    }
    finish_lp(lp);
    return lp;
}

void finish_lp(ConsensusLP& lp) {
    if (lp.n < 1) fail(LDOPF_INVALID_ARGUMENT, "the LP needs at least one global variable");
    if (lp.S < 1) fail(LDOPF_INVALID_ARGUMENT, "the LP needs at least one subsystem");
    if (int64_t(lp.ns.size()) != lp.S || int64_t(lp.ms.size()) != lp.S) fail(LDOPF_INVALID_ARGUMENT, "size arrays do not match S");
    if (int64_t(lp.c.size()) != lp.n || int64_t(lp.lo.size()) != lp.n || int64_t(lp.hi.size()) != lp.n)
        fail(LDOPF_INVALID_ARGUMENT, "global arrays do not match n");
    lp.loc_off.assign(lp.S + 1, 0);
    lp.row_off.assign(lp.S + 1, 0);
    lp.a_off.assign(lp.S + 1, 0);
    for (int64_t s = 0; s < lp.S; ++s) {
        if (lp.ns[s] < 1) fail(LDOPF_INVALID_ARGUMENT, "subsystem " + std::to_string(s) + " has no variables");
        if (lp.ms[s] < 0) fail(LDOPF_INVALID_ARGUMENT, "subsystem " + std::to_string(s) + " has a negative row count");
        lp.loc_off[s + 1] = lp.loc_off[s] + lp.ns[s];
        lp.row_off[s + 1] = lp.row_off[s] + lp.ms[s];
        lp.a_off[s + 1] = lp.a_off[s] + int64_t(lp.ns[s]) * lp.ms[s];
    }
    if (int64_t(lp.gidx.size()) != lp.loc_off[lp.S] || int64_t(lp.b.size()) != lp.row_off[lp.S] ||
        int64_t(lp.A.size()) != lp.a_off[lp.S])
        fail(LDOPF_INVALID_ARGUMENT, "concatenated arrays do not match the subsystem sizes");
    std::vector<int32_t> copies(lp.n, 0);
    for (int64_t s = 0; s < lp.S; ++s)
        for (int64_t k = lp.loc_off[s]; k < lp.loc_off[s + 1]; ++k) {
            const int64_t g = lp.gidx[k];
            if (g < 0 || g >= lp.n) fail(LDOPF_INVALID_ARGUMENT, "gidx out of range");
            if (k > lp.loc_off[s] && g <= lp.gidx[k - 1])
                fail(LDOPF_INVALID_ARGUMENT, "gidx must be strictly ascending inside subsystem " + std::to_string(s));
            copies[g]++;
        }
    for (int64_t g = 0; g < lp.n; ++g) {
        if (copies[g] == 0) fail(LDOPF_INVALID_ARGUMENT, "global variable " + std::to_string(g) + " has no local copy");
        if (std::isnan(lp.c[g]) || std::isnan(lp.lo[g]) || std::isnan(lp.hi[g]) || std::isinf(lp.c[g]))
            fail(LDOPF_INVALID_ARGUMENT, "NaN in c, lo or hi, or infinite c");
        if (lp.lo[g] > lp.hi[g]) fail(LDOPF_INFEASIBLE_BOUNDS, "global variable " + std::to_string(g) + ": lower bound above upper bound");
    }
    for (double v : lp.A)
        if (!std::isfinite(v)) fail(LDOPF_INVALID_ARGUMENT, "non-finite entry in A");
    for (double v : lp.b)
        if (!std::isfinite(v)) fail(LDOPF_INVALID_ARGUMENT, "non-finite entry in b");
    if (lp.x_init.empty()) {
        lp.x_init.resize(lp.n);
        for (int64_t v = 0; v < lp.n; ++v) {
            double s = std::min(std::max(0.0, lp.lo[v]), lp.hi[v]);
            if (std::isfinite(lp.lo[v]) && std::isfinite(lp.hi[v])) s = 0.5 * (lp.lo[v] + lp.hi[v]);
            lp.x_init[v] = s;
        }
    } else {
        if (int64_t(lp.x_init.size()) != lp.n) fail(LDOPF_INVALID_ARGUMENT, "x_init does not match n");
        for (double v : lp.x_init)
            if (!std::isfinite(v)) fail(LDOPF_INVALID_ARGUMENT, "non-finite entry in x_init");
    }
    if (!lp.locality_order.empty() && int64_t(lp.locality_order.size()) != lp.S)
        fail(LDOPF_INVALID_ARGUMENT, "internal: locality order does not cover every subsystem");
}

}  // namespace ldopf
