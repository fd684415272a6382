// Task-graph planner: reduction trees, step sequences, tile dependencies and
// critical paths.  See plan.hpp for the model.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace bb {

const double kTable1Weights[6] = {4.0, 6.0, 2.0, 6.0, 12.0, 6.0};

int auto_domain(int u, int v, int workgroups, double gamma) {
    // Section 5: pick a per step so that ceil(u/a) * v parallel tasks are at
    // least gamma * nb_cores; the largest such a keeps the most TS kernels.
    double need = gamma * (double)workgroups;
    int vv = v > 1 ? v : 1;
    for (int a = u; a >= 1; --a) {
        long long dom = (u + a - 1) / a;
        if ((double)dom * (double)vv >= need) return a;
    }
    return 1;
}

std::vector<Elim> step_tree(int tree, int u, int a) {
    std::vector<Elim> el;
    if (u <= 1) return el;
    switch (tree) {
    case FLATTS:   // Section 3.3: pivot is the diagonal tile, eliminate in order, TS
        for (int i = 1; i < u; ++i) el.push_back({i, 0, 0});
        break;
    case FLATTT:   // same eliminations with TT kernels
        for (int i = 1; i < u; ++i) el.push_back({i, 0, 1});
        break;
    case GREEDY:   // one BiDiag step: binomial tree (Section 3.6), TT kernels
        for (int s = 1; s < u; s *= 2)
            for (int i = s; i < u; i += 2 * s) el.push_back({i, i - s, 1});
        break;
    case AUTO: {   // Section 5: FlatTS domains of size a joined by a Greedy TT tree
        if (a < 1) a = 1;
        int ndom = (u + a - 1) / a;
        for (int d = 0; d < ndom; ++d) {
            int head = d * a;
            int end = std::min(head + a, u);
            for (int i = head + 1; i < end; ++i) el.push_back({i, head, 0});
        }
        for (int s = 1; s < ndom; s *= 2)
            for (int h = s; h < ndom; h += 2 * s) el.push_back({h * a, (h - s) * a, 1});
        break;
    }
    default:
        break;
    }
    return el;
}

namespace {

struct Builder {
    Graph& g;
    int p, q;
    std::vector<int32_t> last_writer;   // per physical tile
    std::vector<int32_t> slot_owner;    // slot -> panel task

    Builder(Graph& gg, int pp, int qq) : g(gg), p(pp), q(qq), last_writer((size_t)pp * qq, -1) {}

    int32_t add(Task t) {
        int32_t id = (int32_t)g.tasks.size();
        std::vector<int32_t> pr;
        auto touch = [&](int r, int c) {
            if (r < 0) return;
            int32_t& w = last_writer[(size_t)r * q + c];
            if (w >= 0) pr.push_back(w);
            w = id;
        };
        touch(t.r1, t.c1);
        touch(t.r2, t.c2);
        if (!is_panel(t.kind)) pr.push_back(slot_owner[t.slot]);
        std::sort(pr.begin(), pr.end());
        pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
        g.tasks.push_back(t);
        g.pred.push_back(std::move(pr));
        return id;
    }

    int32_t new_slot(int32_t owner_task) {
        slot_owner.push_back(owner_task);
        return g.nslots++;
    }

    // One QR step in the logical frame (trans = 1 for LQ): panel tiles
    // (rows[li], kcol), trailing tiles (rows[li], cols[*]).
    struct StepState {
        int trans, kcol, step;
        std::vector<int> rows, cols;
        std::vector<char> tri;
    };

    void phys(int trans, int lr, int lc, int32_t& r, int32_t& c) const {
        if (trans) { r = lc; c = lr; } else { r = lr; c = lc; }
    }

    void ensure_tri(StepState& s, int li) {
        if (s.tri[li]) return;
        Task t{GEQRT, s.trans, 0, 0, -1, -1, 0, s.step};
        phys(s.trans, s.rows[li], s.kcol, t.r1, t.c1);
        int32_t id = (int32_t)g.tasks.size();
        t.slot = new_slot(id);
        add(t);
        for (int c : s.cols) {
            Task u{UNMQR, s.trans, -1, -1, 0, 0, t.slot, s.step};
            phys(s.trans, s.rows[li], c, u.r2, u.c2);
            add(u);
        }
        s.tri[li] = 1;
    }

    void eliminate(StepState& s, const Elim& e) {
        ensure_tri(s, e.piv);
        if (e.tt) ensure_tri(s, e.i);
        Task t{e.tt ? TTQRT : TSQRT, s.trans, 0, 0, 0, 0, 0, s.step};
        phys(s.trans, s.rows[e.piv], s.kcol, t.r1, t.c1);
        phys(s.trans, s.rows[e.i], s.kcol, t.r2, t.c2);
        int32_t id = (int32_t)g.tasks.size();
        t.slot = new_slot(id);
        add(t);
        for (int c : s.cols) {
            Task u{e.tt ? TTMQR : TSMQR, s.trans, 0, 0, 0, 0, t.slot, s.step};
            phys(s.trans, s.rows[e.piv], c, u.r1, u.c1);
            phys(s.trans, s.rows[e.i], c, u.r2, u.c2);
            add(u);
        }
    }

    StepState make_step(int trans, int kcol, int r0, int r1, int c0, int c1) {
        StepState s;
        s.trans = trans;
        s.kcol = kcol;
        s.step = g.nsteps++;
        for (int r = r0; r < r1; ++r) s.rows.push_back(r);
        for (int c = c0; c < c1; ++c) s.cols.push_back(c);
        s.tri.assign(s.rows.size(), 0);
        return s;
    }

    void run_step(int trans, int kcol, int r0, int r1, int c0, int c1) {
        StepState s = make_step(trans, kcol, r0, r1, c0, c1);
        int u = (int)s.rows.size(), v = (int)s.cols.size();
        int a = 0;
        if (g.opt.tree == AUTO)
            a = g.opt.auto_a > 0 ? g.opt.auto_a : auto_domain(u, v, g.opt.workgroups, g.opt.gamma);
        g.auto_a_used.push_back(a);
        for (const Elim& e : step_tree(g.opt.tree, u, a)) eliminate(s, e);
        ensure_tri(s, 0);
    }

    // QR of tile rows j0..pend-1, tile columns j0..q-1 with the Greedy tree
    // over all columns at once (used by R-BiDiag, j0 = 0, and by the
    // three-step reduction).  Synchronous rounds: in column j the rows
    // already zeroed in column j-1 but not yet in column j are candidates;
    // the bottom half of them is eliminated (TT) by the rows just above.
    void greedy_qr(int pend, int j0) {
        std::vector<StepState> cols;
        for (int j = j0; j < q; ++j) cols.push_back(make_step(0, j, j, pend, j + 1, q));
        for (int j = j0; j < q; ++j) g.auto_a_used.push_back(0);
        const int nc = q - j0;
        std::vector<int> nz(nc, 0);
        for (;;) {
            std::vector<int> nzn = nz;
            bool any = false;
            for (int jj = 0; jj < nc; ++jj) {
                const int j = j0 + jj;
                int top = (jj == 0) ? j0 : pend - nz[jj - 1];
                top = std::max(top, j);
                int bottom = pend - nz[jj];
                int z = bottom - top;
                int e = z / 2;
                for (int t = 0; t < e; ++t) {
                    int i = bottom - 1 - t;
                    eliminate(cols[jj], Elim{i - j, i - e - j, 1});
                }
                nzn[jj] += e;
                if (e > 0) any = true;
            }
            nz = nzn;
            if (!any) break;
        }
        for (int jj = 0; jj < nc; ++jj) ensure_tri(cols[jj], 0);
    }

    // R-BiDiag on the trailing tiles (s.., s..): QR of rows s..p-1, columns
    // s..q-1, then the band reduction of the top (q-s) x (q-s) tiles.
    void rbidiag_from(int s, bool qr_only) {
        if (g.opt.tree == GREEDY) {
            greedy_qr(p, s);
        } else {
            for (int k = s; k < q; ++k) run_step(0, k, k, p, k + 1, q);
        }
        if (qr_only) return;
        g.phase2_start = (int32_t)g.tasks.size();
        for (int k = s; k < q; ++k) {
            if (k > s) run_step(0, k, k, q, k + 1, q);       // QR(k) on the top tiles
            if (k + 1 < q) run_step(1, k, k + 1, q, k + 1, q);  // LQ(k)
        }
    }
};

}  // namespace

int three_step_switch(int p, int q, double delta) {
    for (int k = 0; k < q; ++k)
        if ((double)(p - k) >= delta * (double)(q - k)) return k;
    return q;
}

std::string build_graph(int p, int q, const PlanOptions& opt, Graph& g) {
    if (q < 1 || p < q) return "tile grid must satisfy p >= q >= 1";
    if (opt.tree < FLATTS || opt.tree > AUTO) return "unknown tree";
    if (opt.variant < BIDIAG || opt.variant > THREESTEP) return "unknown variant";
    g = Graph();
    g.p = p;
    g.q = q;
    g.opt = opt;
    Builder b(g, p, q);
    // BiDiag steps QR(k); LQ(k) for k < s, then R-BiDiag on what is left
    // (Sections 3.4, 3.5 and 4.5).
    int s = 0;
    switch (opt.variant) {
    case BIDIAG: s = q; break;
    case RBIDIAG: case QRONLY: s = 0; break;
    default: s = opt.switch_step >= 0 ? std::min(opt.switch_step, q) : three_step_switch(p, q, opt.delta); break;
    }
    g.switch_step = s;
    for (int k = 0; k < s; ++k) {
        b.run_step(0, k, k, p, k + 1, q);                     // QR(k)
        if (k + 1 < q) b.run_step(1, k, k + 1, q, k + 1, p);  // LQ(k)
    }
    if (s < q) b.rbidiag_from(s, opt.variant == QRONLY);
    return std::string();
}

std::string check_graph(int p, int q, int64_t nt, const int32_t* tk, const int32_t* off,
                        const int32_t* idx) {
    std::vector<int32_t> last((size_t)p * q, -1), slot_owner;
    auto has_edge = [&](int64_t t, int32_t pr) {
        for (int32_t e = off[t]; e < off[t + 1]; ++e)
            if (idx[e] == pr) return true;
        return false;
    };
    char buf[160];
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* x = tk + 8 * t;
        for (int32_t e = off[t]; e < off[t + 1]; ++e)
            if (idx[e] < 0 || idx[e] >= t) {
                snprintf(buf, sizeof buf, "task %lld: predecessor %d does not precede it", (long long)t, idx[e]);
                return buf;
            }
        const int kind = x[0];
        if (kind < GEQRT || kind > TTMQR) return "unknown task kind";
        const int32_t coords[2][2] = {{x[2], x[3]}, {x[4], x[5]}};
        for (int k = 0; k < 2; ++k) {
            const int r = coords[k][0], c = coords[k][1];
            if (r < 0) continue;
            if (r >= p || c >= q) return "tile out of range";
            int32_t& l = last[(size_t)r * q + c];
            if (l >= 0 && !has_edge(t, l)) {
                snprintf(buf, sizeof buf, "tasks %d and %lld touch tile (%d,%d) without an edge", l, (long long)t, r, c);
                return buf;
            }
            l = (int32_t)t;
        }
        const int32_t slot = x[6];
        if (slot < 0) return "negative slot";
        if (is_panel(kind)) {
            if ((size_t)slot >= slot_owner.size()) slot_owner.resize(slot + 1, -1);
            if (slot_owner[slot] >= 0) return "V/T slot written twice";
            slot_owner[slot] = (int32_t)t;
        } else {
            if ((size_t)slot >= slot_owner.size() || slot_owner[slot] < 0) return "update reads an unwritten slot";
            if (!has_edge(t, slot_owner[slot])) {
                snprintf(buf, sizeof buf, "update %lld does not depend on the panel of its slot", (long long)t);
                return buf;
            }
        }
    }
    return std::string();
}

void build_apply_graph(const Graph& g, int side, int transpose, int jc, Graph& out) {
    const int rows = side == 0 ? g.p : g.q;
    out = Graph();
    out.p = rows;
    out.q = jc;
    out.opt = g.opt;
    out.nslots = g.nslots;
    std::vector<int32_t> panels;
    for (size_t t = 0; t < g.tasks.size(); ++t)
        if (is_panel(g.tasks[t].kind) && g.tasks[t].trans == side) panels.push_back((int32_t)t);
    if (!transpose) std::reverse(panels.begin(), panels.end());
    std::vector<int32_t> last((size_t)rows * jc, -1);
    out.tasks.reserve(panels.size() * (size_t)jc);
    out.pred.reserve(panels.size() * (size_t)jc);
    for (int32_t pt : panels) {
        const Task& x = g.tasks[pt];
        // Rows of C that the reflectors act on: the physical tile rows of a
        // QR-step panel, the physical tile columns of an LQ-step panel.
        const int32_t a1 = side == 0 ? x.r1 : x.c1;
        const int32_t a2 = x.kind == GEQRT ? -1 : (side == 0 ? x.r2 : x.c2);
        const int32_t kind = x.kind + 3 + (transpose ? 0 : APPLY_H);   // GEQRT -> UNMQR, ...
        for (int J = 0; J < jc; ++J) {
            Task u{};
            u.kind = kind;
            u.trans = 0;
            u.slot = x.slot;
            u.step = x.step;
            if (x.kind == GEQRT) {          // UNMQR: C2 is the panel's own tile row
                u.r1 = -1; u.c1 = -1; u.r2 = a1; u.c2 = J;
            } else {
                u.r1 = a1; u.c1 = J; u.r2 = a2; u.c2 = J;
            }
            const int32_t id = (int32_t)out.tasks.size();
            std::vector<int32_t> pr;
            for (int32_t r : {u.r1, u.r2}) {
                if (r < 0) continue;
                int32_t& l = last[(size_t)r * jc + J];
                if (l >= 0) pr.push_back(l);
                l = id;
            }
            std::sort(pr.begin(), pr.end());
            pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
            out.tasks.push_back(u);
            out.pred.push_back(std::move(pr));
        }
    }
}

void append_graph(Graph& g, const Graph& h, int32_t mat) {
    const int32_t t0 = (int32_t)g.tasks.size();
    const int32_t s0 = g.nslots;
    g.p = std::max(g.p, h.p);
    g.q = std::max(g.q, h.q);
    for (size_t t = 0; t < h.tasks.size(); ++t) {
        Task x = h.tasks[t];
        x.slot += s0;
        x.mat = mat;
        g.tasks.push_back(x);
        std::vector<int32_t> pr(h.pred[t]);
        for (int32_t& v : pr) v += t0;
        g.pred.push_back(std::move(pr));
    }
    g.nslots += h.nslots;
    g.nsteps = std::max(g.nsteps, h.nsteps);
}

double critical_path(const Graph& g, const double* w) {
    std::vector<double> fin(g.tasks.size(), 0.0);
    double best = 0.0;
    for (size_t t = 0; t < g.tasks.size(); ++t) {
        double s = 0.0;
        for (int32_t pr : g.pred[t]) s = std::max(s, fin[pr]);
        fin[t] = s + w[g.tasks[t].kind];
        best = std::max(best, fin[t]);
    }
    return best;
}

}  // namespace bb
