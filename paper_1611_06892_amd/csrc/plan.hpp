// Task-graph planner for tiled band bidiagonalization (host side, plain C++).
//
// A p x q tile matrix (tiles nb x nb) is reduced by the step sequences of
// Section 3.4 (BiDiag: QR(1); LQ(1); ...; QR(q)) or Section 3.5 (R-BiDiag:
// QR(p,q) then LQ(1); QR(2); ...; QR(q) on the top q x q tiles).  Each step
// eliminates the tiles of one tile column (QR) or tile row (LQ) along a
// reduction tree (Section 3.3, FlatTS / FlatTT / Greedy; Section 5, Auto),
// using the six kernels of Table 1 (Algorithms 2 and 3).  LQ steps are QR
// steps on the transposed tile matrix (Algorithm 4 and the text after it), so
// every task is described in a "logical" frame and carries a transpose flag.
//
// The planner emits tasks in a valid sequential program order and derives the
// dependencies from tile accesses: every tile access of a kernel is a
// read-modify-write, and reflectors (V, T) go to write-once slots outside the
// matrix, so each task depends on the previous writer of each tile it touches
// and on the panel whose slot it reads.  With Table 1 weights the longest path
// of this graph is the critical path of Section 4.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace bb {

enum Kind : int { GEQRT = 0, TSQRT = 1, TTQRT = 2, UNMQR = 3, TSMQR = 4, TTMQR = 5 };
// Updates that apply H = I - V T V^T itself instead of H^T (blocks of the
// record in reverse order, T instead of T^T): UNMQR + APPLY_H, ...
enum : int { APPLY_H = 3, NKINDS = 9 };
enum Tree : int { FLATTS = 0, FLATTT = 1, GREEDY = 2, AUTO = 3 };
// QRONLY is the tiled QR factorization QR(p,q) of Algorithm 1 alone (the first
// phase of R-BiDiag); it exists for the critical-path formulas of Section 4.3.
// THREESTEP is the three-step reduction of Section 4.5: BiDiag steps
// QR(k); LQ(k) for k < s, then R-BiDiag on the trailing (p-s) x (q-s) tiles
// (s = 0 is R-BiDiag, s = q is BiDiag).
enum Variant : int { BIDIAG = 0, RBIDIAG = 1, QRONLY = 2, THREESTEP = 3 };

inline bool is_panel(int k) { return k <= TTQRT; }

// One kernel invocation.  Tile coordinates are physical (row, column) tile
// indices of the matrix.  For panels, (r1,c1) is the tile that ends up
// triangular (GEQRT: the tile factored; TS/TT: the pivot tile) and (r2,c2) the
// tile that is zeroed (-1 for GEQRT).  For updates, (r1,c1) is the pivot-row
// tile C1 (-1 for UNMQR) and (r2,c2) the tile C2 that receives V * W.
struct Task {
    int32_t kind;
    int32_t trans;   // 0: QR step (left, on columns); 1: LQ step (right, on rows)
    int32_t r1, c1, r2, c2;
    int32_t slot;    // V/T slot written (panel) or read (update)
    int32_t step;    // index of the QR/LQ step this task belongs to
    int32_t mat;     // matrix of a batched graph (0 otherwise)
};

struct PlanOptions {
    int tree = AUTO;
    int variant = BIDIAG;
    int workgroups = 256;   // concurrent workers assumed by Auto (nb_cores in Section 5)
    double gamma = 2.0;     // Auto's parallelism factor (Section 5 uses 2)
    int auto_a = 0;         // > 0 forces the FlatTS domain size of Auto
    int switch_step = -1;   // THREESTEP: the step s; < 0 chooses it by delta
    double delta = 5.0;     // THREESTEP: switch once the trailing tiles have p - k >= delta (q - k)
};

// THREESTEP's switch step for a p x q tile matrix: the first k with
// p - k >= delta (q - k) (the trailing matrix is then tall enough for
// R-BiDiag to have the shorter critical path, Sections 4.3.4 and 4.5), else q.
int three_step_switch(int p, int q, double delta);

struct Graph {
    int p = 0, q = 0;
    PlanOptions opt;
    std::vector<Task> tasks;                 // program order (a topological order)
    std::vector<std::vector<int32_t>> pred;  // distinct predecessors
    int32_t nslots = 0;                      // V/T slots (one per panel task)
    int32_t nsteps = 0;
    std::vector<int32_t> auto_a_used;        // per step (Auto), for inspection
    int32_t phase2_start = -1;               // R-BiDiag: first task of the band reduction of R
    int32_t switch_step = -1;                // THREESTEP: the step s used
};

// Build the task graph.  Returns an empty string on success, else a message.
std::string build_graph(int p, int q, const PlanOptions& opt, Graph& g);

// Table 1 weights in units of nb^3/3 flops: GEQRT 4, TSQRT 6, TTQRT 2,
// UNMQR 6, TSMQR 12, TTMQR 6.
extern const double kTable1Weights[6];

// Graph that applies the reflectors recorded by a reduction graph g to a
// matrix C whose rows are the tile rows (side 0, Q) or the tile columns
// (side 1, P) of the reduced matrix, with jc tile columns.  The forward
// applies H_1^T, H_2^T, ... (panels in program order), so Q = H_1 H_2 ... over
// the QR-step panels (trans 0) and P = G_1 G_2 ... over the LQ-step panels
// (trans 1), with B = Q^T A P (Sections 3.4, 3.5).  transpose = 1 builds
// C <- Q^T C (P^T C): every panel's update in program order;  transpose = 0
// builds C <- Q C (P C): the panels in reverse order with APPLY_H kinds.
// Tasks carry trans 0 (C is not transposed) and the panel's slot; each
// depends on the previous task that touched one of its C tiles.
void build_apply_graph(const Graph& g, int side, int transpose, int jc, Graph& out);

// Appends graph h (of matrix `mat`) to the union graph g of a batch: task
// indices, predecessors and slots are offset; no edge joins two matrices.
void append_graph(Graph& g, const Graph& h, int32_t mat);

// Static race check of a task graph given as arrays (program order):
// predecessors precede their task; every two consecutive tasks touching the
// same tile are ordered by an edge (all tile accesses are read-modify-write,
// so this orders every conflicting pair); every update depends on the panel
// that wrote its V/T slot, which is written by exactly one panel.  Returns an
// empty string when the graph is race-free, else a description.
std::string check_graph(int p, int q, int64_t ntasks, const int32_t* tasks,
                        const int32_t* pred_off, const int32_t* pred_idx);

// Longest weighted path (critical path, Section 4) with per-kind weights.
double critical_path(const Graph& g, const double* weights);

// Elimination list of one step on u panel tiles (local index 0 = diagonal
// tile).  Each entry (i, piv, tt) zeroes local tile i against local tile piv
// with TS (tt = 0) or TT (tt = 1) kernels, in a valid sequential order.
struct Elim { int32_t i, piv, tt; };
std::vector<Elim> step_tree(int tree, int u, int a);

// Auto's domain size for a step with u panel tiles and v trailing tiles:
// the largest a in [1,u] with ceil(u/a) * max(v,1) >= gamma * workgroups,
// else 1 (Section 5).
int auto_domain(int u, int v, int workgroups, double gamma);

}  // namespace bb
