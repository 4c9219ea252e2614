/*
 * libpf: Newton-Raphson AC power flow on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem (Shi et al.,
 * "Graph Based Power Flow Calculation for Energy Management System",
 * arXiv 1811.02512): a grid graph with admittances on edges and shunts on
 * nodes (Sec. III-A) -> form the admittance matrix (FormMatrixA) -> analyse
 * the sparsity (FormFilledGraph, FormEliminationTree,
 * FormHierarchicalPartition; Sec. II-B) -> factorise A = LDU level by level
 * (FactorizeGraphA, Sec. III-B) -> forward substitution, normalisation and
 * backward substitution (Sec. III-C), all inside Newton-Raphson (Sec. III).
 *
 * Conventions shared by every call
 *   - Buses are numbered 0..n-1; one bus is the slack (reference) bus.
 *   - Per-unit quantities, angles in radians, fp64 everywhere.
 *   - Bus types: PF_BUS_PQ, PF_BUS_PV, PF_BUS_SLACK (int8).  Any type other
 *     than PF_BUS_PV at a non-slack bus is treated as PQ; the slack is the
 *     one named to pf_analyze.
 *   - "Position" p = 0..nn-1 (nn = n-1) is the elimination position of a
 *     non-slack bus; perm[p] is its bus.
 *   - A 2x2 block is 4 doubles row-major [r0c0 r0c1 r1c0 r1c1]; row 0 is the
 *     active-power equation, row 1 the reactive-power equation (PQ bus) or
 *     the |V| equation (PV bus); column 0 is the angle unknown, column 1 the
 *     magnitude unknown.  A PV bus keeps |V| fixed: its row-1 block entries
 *     are (0,1) on the diagonal and (0,0) elsewhere, and its column-1 entries
 *     off its own row are zero.
 *   - Filled layout ("vals"), per case, lu_offset + 8*nnzL doubles with
 *     lu_offset = 8*ceil(nn/2) (info.lu_offset):
 *       D section  [nn][4]        diagonal block of position p, then zero
 *                                 padding up to lu_offset (so that every
 *                                 slot record starts on a 64-byte boundary)
 *       LU section [nnzL][2][4]   at lu_offset: for slot s of S(p) (the s-th higher
 *                                 neighbour k of p in the filled graph):
 *                                 [0] = block (k, p) below the diagonal,
 *                                 [1] = block (p, k) above it.
 *     After pf_factor the same layout holds the factors: D section = D^-1,
 *     LU[s][0] = L_kp * D_p (lower factor times pivot), LU[s][1] = U_pk (unit
 *     upper factor), so that A = L D U with L, U unit block-triangular.
 *   - Device pointers are caller-owned (e.g. torch tensors) and must stay
 *     valid until the stream work completes.  libpf allocates no device
 *     memory; pf_symbolic_upload / pf_multi_upload copy into caller buffers.
 *   - "stride" arguments are in elements between consecutive cases; 0 means
 *     the array is shared by all cases (inputs only).  With B > 1 any other
 *     stride must be at least the array's row (nnz_y pairs for admittance
 *     values, n for bus arrays, m for branch arrays, 2 nn for mismatch and
 *     adjoint vectors): a smaller one returns PF_E_WORKSPACE, a negative
 *     one PF_E_INVALID or PF_E_WORKSPACE, in both cases before any launch.
 *   - Interleaved case groups ("interleave" C in 1, 2, 4, 8): an array of
 *     per-case doubles with stride S (a multiple of 8) is cut into groups of
 *     C cases; element d of case c lives at
 *       (c / C) * C * S + (d / 8) * 8 C + 8 (c % C) + d % 8,
 *     i.e. the 64-byte chunks (one slot record, two D blocks) of the C cases
 *     of a group alternate: a case's record stays in one 128-byte line, and
 *     a line carries the same record of two cases.  (pf_newton's own part of
 *     the workspace after the filled values, its bus records and rhs, is
 *     internal; it is interleaved in 32-byte chunks.)
 *     The buffer holds ceil(B / C) * C * S doubles.  C = 1 is the plain
 *     [B][S] layout.  Kernels launch the C workgroups of a group 8 blocks
 *     apart, which puts them on the same XCD of the MI355X at the same time,
 *     so the cases of a group share each fetched line through that L2.
 *   - Every stream argument is a hipStream_t (0 = legacy default stream);
 *     work is enqueued asynchronously, so per-case numerical outcomes are
 *     reported in device status arrays, never by the return code.
 *   - Return codes (pf_status) report argument, analysis and launch errors
 *     synchronously; pf_last_error() gives a thread-local message.
 *   - No C++ exception crosses this interface.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_symbolic_s* pf_symbolic;
typedef struct pf_multi_s* pf_multi;

typedef enum {
    PF_OK = 0,
    PF_E_INVALID = 1,       /* bad argument, bad branch list, self loop       */
    PF_E_HIP = 2,           /* a HIP runtime call failed                     */
    PF_E_WORKSPACE = 3,     /* caller buffer too small / misaligned          */
    PF_E_DISCONNECTED = 4,  /* some bus is not connected to the slack        */
    PF_E_ZERO_PIVOT = 5,    /* per case: singular or non-finite pivot block  */
    PF_E_NOT_CONVERGED = 6, /* per case: max_iter reached                    */
    PF_E_NONFINITE = 7      /* per case: NaN/Inf mismatch                    */
} pf_status;

enum { PF_ORDER_MINDEG = 0, PF_ORDER_NATURAL = 1 };
enum { PF_BUS_PQ = 1, PF_BUS_PV = 2, PF_BUS_SLACK = 3 };
/* pf_newton flags */
enum {
    PF_NEWTON_KEEP_FACTORS = 1 /* after convergence, factor J at the returned
                                  state into the workspace's vals region */
};

typedef struct {
    int32_t n;            /* buses                                          */
    int32_t m;            /* branches                                       */
    int32_t nn;           /* positions (non-slack buses) = n - 1            */
    int32_t slack;
    int64_t nnz_y;        /* admittance entries (diagonal always present)   */
    int64_t nnz_l;        /* off-diagonal blocks of L (= of U)              */
    int64_t n_upd;        /* off-diagonal block updates per factorisation   */
    int32_t nlevels;      /* hierarchical levels                            */
    int32_t max_level_width;
    int64_t vals_doubles;    /* lu_offset + 8*nnz_l: filled layout, one case */
    int64_t ws_doubles;      /* pf_newton workspace per case (vals first)   */
    size_t dev_bytes;        /* device buffer for pf_symbolic_upload        */
    int32_t tail_levels;     /* top levels factorised and solved in LDS     */
    int32_t tail_nodes;
    int32_t tail_lds_bytes;  /* dynamic LDS per workgroup for the tail      */
    int32_t threads;         /* workgroup size, 0 = chosen per launch       */
    int32_t tail_clique;     /* top nodes of the tail handled as a dense     */
                             /* clique (right-looking, one barrier a pivot) */
    int32_t ws_interleave;   /* cases per interleaved group in pf_newton's   */
                             /* workspace (1, 2, 4 or 8)                   */
    int64_t lu_offset;       /* doubles before the LU section (8*ceil(nn/2)) */
    int64_t fd_mat_doubles;  /* fast decoupled B' and B'' of one case        */
    int64_t fd_ws_doubles;   /* pf_fdpf workspace per case                   */
    int32_t spread;          /* workgroups of a one-case pf_newton launch    */
                             /* (0: one workgroup)                          */
    int32_t sub_levels;      /* bottom levels that the groups of a spread    */
                             /* batch of grids (pf_multi_set_spread) run as */
                             /* whole subtrees per workgroup, without grid  */
                             /* barriers (0: none)                          */
} pf_info;

/* ---- status ------------------------------------------------------------ */
const char* pf_status_string(int status);
/* Last error message of the calling thread ("" if none). */
const char* pf_last_error(void);
const char* pf_version(void);

/* ---- symbolic analysis (host, synchronous, no GPU needed) ---------------
 * Paper: FormFilledGraph, FormEliminationTree and FormHierarchicalPartition
 * (Sec. II-B) on the bus graph without the slack.  The paper eliminates in
 * the given numbering; ordering PF_ORDER_MINDEG (default) first applies an
 * exact minimum-degree order (degree = distinct uneliminated neighbours with
 * fill; ties to the lowest bus number), PF_ORDER_NATURAL keeps bus order.
 * Levels: synchronous leaf peeling of the elimination tree (Table I); nodes
 * of a level are listed in ascending position.
 * from/to: host int32[m]; parallel branches allowed; self loops rejected.
 * Errors: PF_E_INVALID (n < 2, index out of range, self loop, bad slack),
 * PF_E_DISCONNECTED (a bus unreachable from the slack).  On success *out
 * owns a host object; release it with pf_symbolic_destroy.               */
int pf_analyze(int n, int m, const int32_t* from, const int32_t* to, int slack,
               int ordering, pf_symbolic* out);
int pf_symbolic_info(const pf_symbolic sym, pf_info* info);
/* Copies the analysis into caller host arrays: perm[nn] (bus at position p),
 * parent[nn] (elimination-tree parent position, -1 for roots), level[nn]
 * (1-based), level_ptr[nlevels+1], level_nodes[nn], Lp[nn+1], Li[nnz_l]
 * (S(p) = Li[Lp[p]..Lp[p+1]), ascending).  Any pointer may be NULL.       */
int pf_symbolic_export(const pf_symbolic sym, int32_t* perm, int32_t* parent,
                       int32_t* level, int32_t* level_ptr, int32_t* level_nodes,
                       int32_t* Lp, int32_t* Li);
/* Thread mapping: lanes per node (1,2,4,...,64) for each level, used by the
 * level-scheduled kernels.  Defaults come from a work model; an autotuner may
 * replace them.  Takes effect at the next pf_symbolic_upload.             */
int pf_symbolic_set_mapping(pf_symbolic sym, const int32_t* lanes_per_level);
/* Launch shape of the level-scheduled kernels: threads per workgroup (64,
 * 128, 256 or 512; 0 = by batch size: 512 up to 512 cases, else 256) and the LDS
 * budget in bytes of the tail, the largest run of top levels whose values
 * (64 bytes per filled slot, 48 per node) are factorised and solved in LDS
 * (0 = none, at most 161792 so that 2 KB of LDS stay for reductions;
 * default 65536).  The Newton kernel's LDS copy of every bus's (e, f)
 * (16 n bytes) is used only when it fits this budget too, so a budget of
 * at most half the LDS lets two workgroups share a CU.  A new budget rebuilds the
 * tail and requires pf_symbolic_upload again.  interleave (1, 2, 4, 8;
 * default 4) is the case grouping of pf_newton's workspace.               */
int pf_symbolic_set_launch(pf_symbolic sym, int threads, int64_t tail_lds_budget,
                           int interleave);
/* Workgroups a one-case pf_newton or pf_newton_noalloc launch spreads over
 * (0 or 1: one workgroup, the default; at most 1024).  With more than one,
 * the loops over buses and the levels below the LDS tail are shared out
 * among that many workgroups of a cooperative launch, which meet at grid
 * barriers, while the tail runs on the first (the paper's nodal parallelism
 * across the device for one case, Sec. III); the count is capped by the
 * workgroups the device keeps resident at once.  Results equal the
 * one-workgroup path's to rounding: the arithmetic of every node is the
 * same, but |V| is read from the bus record rather than recomputed from
 * (e, f).  A launch recorded into a graph (stream capture) and every batch
 * (B > 1) use the one-workgroup kernel.  Takes effect at the next call.    */
int pf_symbolic_set_spread(pf_symbolic sym, int workgroups);
/* The longest wait at a grid barrier of a spread launch before it gives up
 * (every workgroup then stops waiting and runs to its end, and the case
 * reports PF_E_HIP), in ticks of the device's 100 MHz constant clock;
 * default 100000000 (one second).  Tests lower it to exercise that path.  */
int pf_symbolic_set_spread_wait(pf_symbolic sym, uint64_t ticks);
int pf_symbolic_get_mapping(const pf_symbolic sym, int32_t* lanes_per_level);
/* Copies the integer structure into the caller's device buffer d_buf
 * (>= info.dev_bytes, 256-byte aligned) on stream s.  The buffer must stay
 * alive while any call uses this symbolic.  Re-uploading is allowed.    */
int pf_symbolic_upload(pf_symbolic sym, void* d_buf, size_t bytes, void* stream);
void pf_symbolic_destroy(pf_symbolic sym);

/* ---- FormMatrixA (Sec. III-A: admittances on edges, shunts on vertices) --
 * One thread per (case, bus) gathers its row from its shunt and incident
 * branches: Y_ii = y_sh,i + sum (y_e + j b_e/2), Y_ik = -sum y_e,
 * y_e = 1/(r_e + j x_e); parallel branches are summed in branch order.
 * d_r, d_x, d_b: double[B][m] with branch_stride (0 = shared, else >= m).
 * d_ysh: bus shunts y_sh = g + jb as (g, b) pairs, double[B][n][2] with
 * ysh_stride in doubles (0 = shared, else even and >= 2n), 16-byte
 * aligned; NULL = no shunts.
 * d_yval: out, complex as (G, B) pairs, double[B][nnz_y][2] with y_stride
 * (in doubles, >= 2*nnz_y), entries in the symbolic's CSR order.
 * Errors: PF_E_INVALID (NULL array, negative or odd stride, misaligned
 * d_ysh), PF_E_WORKSPACE (a stride too small for B > 1).                */
int pf_build_ybus(const pf_symbolic sym, int B, const double* d_r, const double* d_x,
                  const double* d_b, int64_t branch_stride, const double* d_ysh,
                  int64_t ysh_stride, double* d_yval, int64_t y_stride, void* stream);
/* Copies the admittance CSR structure to host arrays yptr[n+1], ycol[nnz_y]. */
int pf_symbolic_ybus_pattern(const pf_symbolic sym, int32_t* yptr, int32_t* ycol);

/* ---- nodal mismatch (Sec. II-A) -------------------------------------------
 * P_i + jQ_i = V_i conj(sum_k Y_ik V_k); F = calculated - scheduled.
 * d_rhs: out double[B][nn][2] (rhs_stride), position order, (F_P, F_Q) with
 * F_Q = 0 at PV buses.  d_norm: out double[B], max |F| (NaN if any NaN).
 * d_PQ: optional out double[B][n][2] (P_i, Q_i per bus, stride 2n).       */
int pf_mismatch(const pf_symbolic sym, int B, const double* d_yval, int64_t y_stride,
                const int8_t* d_type, int64_t type_stride, const double* d_Psp,
                const double* d_Qsp, int64_t inj_stride, const double* d_Vm,
                const double* d_Va, int64_t v_stride, double* d_rhs, int64_t rhs_stride,
                double* d_norm, double* d_PQ, void* stream);

/* ---- Jacobian ("A matrix formation", Sec. III) ----------------------------
 * Assembles J = dF/d(theta, |V|) of the non-slack buses into the filled
 * layout d_vals (vals_stride >= info.vals_doubles, a multiple of 8); fill
 * slots and the D padding are zero.                                       */
int pf_jacobian(const pf_symbolic sym, int B, const double* d_yval, int64_t y_stride,
                const int8_t* d_type, int64_t type_stride, const double* d_Vm,
                const double* d_Va, int64_t v_stride, double* d_vals, int64_t vals_stride,
                int vals_interleave, void* stream);

/* ---- FactorizeGraphA (Sec. III-B, eqs. 1-3) --------------------------------
 * In-place block LDU of B matrices in the filled layout, level by level
 * (hierarchical parallel), nodes of a level in parallel (nodal parallel).
 * Each node pulls the updates of its descendants (no atomics, results are
 * bitwise reproducible).  No pivoting (Sec. III-B divides by the pivot as
 * it stands): d_status[b] (int32, may be NULL) is set to PF_OK, or to
 * PF_E_ZERO_PIVOT when a pivot block's determinant is zero or not finite;
 * d_pivot[b] (int32, may be NULL) to -1, or to the position of the first
 * failing pivot in the order of a sequential factorisation over the
 * partition (level by level, positions ascending within a level).  The
 * failing pivot's descendants in the tree are still factorised; what
 * follows it is not finite.                                              */
int pf_factor(const pf_symbolic sym, int B, double* d_vals, int64_t vals_stride,
              int vals_interleave, int32_t* d_status, int32_t* d_pivot, void* stream);

/* ---- forward substitution, normalisation, backward substitution ---------
 * (Sec. III-C, eq. 4.)  transpose = 0 solves A x = rhs; transpose = 1 solves
 * A^T x = rhs with the same factors (U^T forward over levels 1..p, D^-T,
 * L^T backward over levels p..1).  d_vals: factored filled layout.  d_rhs:
 * double[B][nn][2] (position order), overwritten with the solution.       */
int pf_solve(const pf_symbolic sym, int B, const double* d_vals, int64_t vals_stride,
             int vals_interleave, double* d_rhs, int64_t rhs_stride, int transpose,
             void* stream);

/* ---- Newton-Raphson (Sec. III) ---------------------------------------------
 * One launch runs the whole iteration for B cases sharing this symbolic;
 * workgroup b owns case b: mismatch, then one sweep over levels 1..p that
 * assembles J, factorises and forward-substitutes, then one sweep p..1 that
 * back-substitutes and applies the step (theta -= dtheta, |V| -= d|V| at PQ
 * buses).  Stops when max|F| < tol at the top of an iteration, or after
 * max_iter steps.  d_Vm/d_Va: in = start state (flat start is the caller's),
 * out = solution, double[B][n] (v_stride).  d_ws: workspace in groups of
 * C = pf_newton_interleave(sym, B) cases (see "Interleaved case groups"), ws_stride
 * >= info.ws_doubles and a multiple of 8, 16-byte aligned (a one-case launch
 * spread over several workgroups, pf_symbolic_set_spread, keeps its
 * grid-barrier words in the last 384 bytes of the case's row).  With
 * PF_NEWTON_KEEP_FACTORS, each converged case's first info.vals_doubles hold
 * the factors of J at the returned state in the filled layout (D^-1, L D,
 * U), so pf_solve and pf_adjoint can take d_ws with vals_stride = ws_stride
 * and vals_interleave = C.  Without the flag, or for a case that did not end
 * PF_OK, that region holds intermediate values only (the iterations keep
 * neither D^-1 nor the top levels' factors there).  Outputs: d_iters[B]
 * (steps applied), d_norm[B] (last max|F|), d_status[B] (PF_OK,
 * PF_E_ZERO_PIVOT, PF_E_NOT_CONVERGED, PF_E_NONFINITE), d_pivot[B] (-1, or
 * with PF_E_ZERO_PIVOT the position of the first failing pivot, as
 * pf_factor); any may be NULL.  The launch never fails because of one case.
 * A spread launch whose workgroups lose step (one of them waits more than a
 * second at a grid barrier) ends every workgroup early and reports
 * PF_E_HIP in d_status.                                                    */
int pf_newton(const pf_symbolic sym, int B, const double* d_yval, int64_t y_stride,
              const int8_t* d_type, int64_t type_stride, const double* d_Psp,
              const double* d_Qsp, int64_t inj_stride, double* d_Vm, double* d_Va,
              int64_t v_stride, double tol, int max_iter, int flags, double* d_ws,
              int64_t ws_stride, int32_t* d_iters, double* d_norm, int32_t* d_status,
              int32_t* d_pivot, void* stream);

/* ---- pf_newton without a workspace argument --------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * launch as pf_newton with flags 0, its workspace taken from a scratch array
 * of PF_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call allocates nothing.  Inputs and outputs
 * as pf_newton.  The batch's workspace, ceil(B / C) * C * info.ws_doubles
 * doubles with C = pf_newton_interleave(sym, B), must fit the array (about
 * 24 cases of 10,000 buses, 140 of 2,000); a larger batch returns
 * PF_E_WORKSPACE before any launch.  Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other streams or
 * threads) race and give wrong results.  Factors are not kept (no
 * PF_NEWTON_KEEP_FACTORS): the array is overwritten by the next call.
 * PF_E_HIP if the array's device address cannot be taken.                 */
#define PF_NOALLOC_SCRATCH_BYTES (64ll << 20)
int pf_newton_noalloc(const pf_symbolic sym, int B, const double* d_yval, int64_t y_stride,
                      const int8_t* d_type, int64_t type_stride, const double* d_Psp,
                      const double* d_Qsp, int64_t inj_stride, double* d_Vm, double* d_Va,
                      int64_t v_stride, double tol, int max_iter, int32_t* d_iters,
                      double* d_norm, int32_t* d_status, int32_t* d_pivot, void* stream);

/* Case grouping pf_newton uses for a batch of B: info.ws_interleave halved
 * until it does not exceed B (1 for a single case).  Returns -1 on error.  */
int pf_newton_interleave(const pf_symbolic sym, int B);

/* ---- fast decoupled power flow (Sec. III; Table III) -----------------------
 * XB scheme (our reading; the paper fixes none): B' from branch reactances
 * only (b'_ik = -sum 1/x over branches i-k, b'_ii = sum 1/x over branches at
 * i), B'' = -Im(Y) of the pi-model with r, x and charging.  Both symmetric,
 * so the factorisation is the paper's LDL^T (eqs. 1-3) with scalar elements
 * on the same filled graph, elimination tree and levels as NR.
 * Matrix layout per case (info.fd_mat_doubles = 2 * M): B' at 0, B'' at M,
 * each d [round8(nn)] (diagonal by position, zero padded) then (lo, up) per
 * slot of S(p) (the symmetric pair of entries).  A PV bus's B'' row and
 * column are the identity.  After pf_fdpf_factor: d = 1/d_j, lo = l_kj d_j,
 * up = l_kj (unit upper factor u_jk = l_kj, eq. 2).
 * pf_fdpf_matrices: branch arrays as pf_build_ybus; d_type int8[B][n];
 * d_mat 16-byte aligned, mat_stride a multiple of 8 (>= fd_mat_doubles if
 * B > 1).  Bus shunts d_ysh as pf_build_ybus (NULL = none): B'' takes
 * -b_sh on its diagonal (B' takes none).  pf_fdpf_factor: in place;
 * d_status[B] (may be NULL) PF_OK or PF_E_ZERO_PIVOT.  Matrices and factors
 * depend on r, x, b, the shunts and the bus types only, so a batch of
 * scenarios shares one (mat_stride = 0).                                   */
int pf_fdpf_matrices(const pf_symbolic sym, int B, const double* d_r, const double* d_x,
                     const double* d_b, int64_t branch_stride, const double* d_ysh,
                     int64_t ysh_stride, const int8_t* d_type, int64_t type_stride,
                     double* d_mat, int64_t mat_stride, void* stream);
int pf_fdpf_factor(const pf_symbolic sym, int B, double* d_mat, int64_t mat_stride,
                   int32_t* d_status, void* stream);

/* One launch runs the decoupled iteration for B cases, one workgroup per
 * case, with the factors of pf_fdpf_factor (mat_stride = 0: shared): with
 * F = calculated - scheduled as for pf_newton, repeat { stop if max|F| < tol;
 * theta -= B'^-1 (F_P / |V|); stop if max|F| < tol; |V| -= B''^-1 (F_Q / |V|)
 * at PQ buses }.  d_iters counts angle half steps, max_iter bounds them.
 * d_ws: ws_stride >= info.fd_ws_doubles (a multiple of 8), 16-byte aligned.
 * d_Vm/d_Va in/out and the outputs as pf_newton (status PF_OK,
 * PF_E_NOT_CONVERGED or PF_E_NONFINITE).                                   */
int pf_fdpf(const pf_symbolic sym, int B, const double* d_yval, int64_t y_stride,
            const int8_t* d_type, int64_t type_stride, const double* d_Psp, const double* d_Qsp,
            int64_t inj_stride, double* d_Vm, double* d_Va, int64_t v_stride,
            const double* d_mat, int64_t mat_stride, double tol, int max_iter, double* d_ws,
            int64_t ws_stride, int32_t* d_iters, double* d_norm, int32_t* d_status,
            void* stream);

/* ---- branch flows (Sec. II-A: post-convergence, nodal/edge parallel) -------
 * For every branch e (from f to t, the analysis' order) of B cases: with
 * y = 1/(r + jx) and charging b, I_ft = (y + jb/2) V_f - y V_t and
 * S_ft = V_f conj(I_ft) = Pft + j Qft, and the same from the to end.  Branch
 * arrays as pf_build_ybus; d_Vm/d_Va double[B][n] (v_stride); outputs
 * double[B][m] (out_stride).                                              */
int pf_branch_flows(const pf_symbolic sym, int B, const double* d_r, const double* d_x,
                    const double* d_b, int64_t branch_stride, const double* d_Vm,
                    const double* d_Va, int64_t v_stride, double* d_Pft, double* d_Qft,
                    double* d_Ptf, double* d_Qtf, int64_t out_stride, void* stream);

/* ---- WLS state estimation ---------------------------------------------------
 * Sec. IV lists state estimation among the applications run on the same
 * graph machinery; the paper gives no formulation, so this is the textbook
 * weighted-least-squares estimator (our reading).  Measurements
 * z = h(x) + e, kind PF_MEAS_*: |V_i|, P_i, Q_i (bus loc), P_ft, Q_ft (flow
 * at the from end of branch loc), weights w = 1/sigma^2.  State x = (theta
 * of every bus but the reference (the slack argument), |V| of every bus).
 * Gauss-Newton: G dx = H^T W (z - h(x)), G = H^T W H, x += dx, until the
 * step's max|dx| < tol.  G is a 2x2 block per pair of buses that share a
 * measurement; pf_se_analyze runs the library's analysis (minimum degree,
 * filled graph, elimination tree, levels) on that graph and plans the
 * assembly; each step assembles G in the filled layout, then runs the
 * pf_factor and pf_solve kernels on it.
 * pf_se_analyze: host arrays (network as pf_analyze; kind int8[M], loc
 * int32[M]); PF_E_INVALID on bad input, PF_E_DISCONNECTED when the
 * measurements leave buses unobservable.  pf_se_upload as
 * pf_symbolic_upload (info.dev_bytes, 256-byte aligned).                   */
enum { PF_MEAS_VM = 1, PF_MEAS_P = 2, PF_MEAS_Q = 3, PF_MEAS_PF = 4, PF_MEAS_QF = 5 };
typedef struct pf_se_s* pf_se;
typedef struct {
    int32_t n, m;
    int32_t measurements;
    int64_t partials;        /* entries of H (measurement, support bus) pairs */
    int64_t gain_nnz_l;      /* off-diagonal blocks of the factored G       */
    int32_t gain_levels;
    int64_t contributions;   /* (measurement, bus pair) terms of G           */
    int64_t ws_doubles;      /* pf_se_estimate scratch per case (see there)  */
    size_t dev_bytes;
} pf_se_dims;
int pf_se_analyze(int n, int m, const int32_t* from, const int32_t* to, int slack, int M,
                  const int8_t* kind, const int32_t* loc, pf_se* out);
int pf_se_info(const pf_se se, pf_se_dims* info);
int pf_se_upload(pf_se se, void* d_buf, size_t bytes, void* stream);
/* Launch shape of the gain matrix's factor and solve kernels (threads and
 * LDS tail budget as pf_symbolic_set_launch); call before pf_se_upload (the
 * upload size changes with the tail).                                      */
int pf_se_set_launch(pf_se se, int threads, int64_t tail_lds_budget);
/* B cases: branch arrays and bus shunts as pf_build_ybus (the injection
 * measurements include the shunts' currents); d_z, d_w double[B][M] (z_stride,
 * w_stride; 0 = shared); d_Vm/d_Va in = start, out = estimate (v_stride);
 * d_ws: scratch of at least ceil(B/4)*4 * ws_doubles doubles, 16-byte
 * aligned (ws_size = doubles available), its layout internal; d_iters,
 * d_norm (last max|dx|), d_status[B] (PF_OK, PF_E_NOT_CONVERGED,
 * PF_E_NONFINITE, the latter also for a singular gain matrix).  The host
 * waits for the stream once per Gauss-Newton step to stop when every case
 * has finished.                                                            */
int pf_se_estimate(const pf_se se, int B, const double* d_r, const double* d_x,
                   const double* d_b, int64_t branch_stride, const double* d_ysh,
                   int64_t ysh_stride, const double* d_z,
                   int64_t z_stride, const double* d_w, int64_t w_stride, double* d_Vm,
                   double* d_Va, int64_t v_stride, double tol, int max_iter, double* d_ws,
                   int64_t ws_size, int32_t* d_iters, double* d_norm, int32_t* d_status,
                   void* stream);
void pf_se_destroy(pf_se se);

/* ---- adjoint right-hand side (beyond the paper) ----------------------------
 * Gathers the loss gradient with respect to the state into position order:
 * d_rhs[b][p] = (dL/dtheta, dL/d|V|) of bus perm[p], with the |V| entry set
 * to zero at PV buses (|V| is fixed there).  d_gVm, d_gVa: double[B][n]
 * (v_stride); d_rhs: out double[B][nn][2] (rhs_stride).                    */
int pf_adjoint_rhs(const pf_symbolic sym, int B, const double* d_gVm, const double* d_gVa,
                   int64_t v_stride, const int8_t* d_type, int64_t type_stride, double* d_rhs,
                   int64_t rhs_stride, void* stream);

/* ---- adjoint parameter gradients (beyond the paper) ------------------------
 * Given lam = J^-T g at the solution (pf_solve with transpose = 1 on the
 * factors kept by pf_newton), writes dL/dPsp = lam_P at non-slack buses,
 * dL/dQsp = lam_Q at PQ buses (0 elsewhere), and
 * dL/dx_e = -sum_{i in {f,t}} lam_i . d(P_i, Q_i)/dx_e, with
 * dy_e/dx_e = -j y_e^2 (r_e held fixed).  d_lam: double[B][nn][2].
 * d_gP, d_gQ: out double[B][n] (g_stride).  d_gx: out; gx_mode 0 writes
 * double[B][m] (stride m), gx_mode 1 writes the sum over cases, double[m].
 * One thread per branch: no atomics.  Errors: PF_E_INVALID (NULL input, bad
 * mode, negative stride, d_gx without d_r and d_x), PF_E_WORKSPACE (with
 * B > 1, a stride below its row: lam 2 nn, Vm/Va and gP/gQ n, a non-zero
 * type stride n, a non-zero branch stride m).                             */
int pf_adjoint_params(const pf_symbolic sym, int B, const double* d_lam, int64_t lam_stride,
                      const int8_t* d_type, int64_t type_stride, const double* d_Vm,
                      const double* d_Va, int64_t v_stride, const double* d_r,
                      const double* d_x, int64_t branch_stride, double* d_gP, double* d_gQ,
                      int64_t g_stride, double* d_gx, int gx_mode, void* stream);

/* ---- fused adjoint backward (beyond the paper) -----------------------------
 * The three steps above in one launch (two with gx_mode 1), on the factors
 * pf_newton kept at the solution (PF_NEWTON_KEEP_FACTORS; d_ws and ws_stride
 * as given to pf_newton with the same B, so the same case grouping): per
 * case, the gradient g = (dL/dtheta, dL/d|V|) gathered into position order
 * (the |V| entry zero at PV buses; d_gVm or d_gVa NULL = zero), the
 * transposed solves J^T lam = g, d_lam <- lam (double[B][nn][2],
 * lam_stride), d_gP, d_gQ (double[B][n], g_stride) as pf_adjoint_params;
 * then d_gx (d_x, d_r and gx_mode as pf_adjoint_params; d_gx NULL =
 * skipped), bit for bit as pf_adjoint_params computes it.  The workspace's
 * bus-record and rhs sections serve as scratch for the branch gradients
 * (overwritten); its factors are left as they are, so pf_adjoint may be
 * called again on the same workspace.  d_status: the per-case status
 * pf_newton wrote, or NULL; a case whose status is not PF_OK (its workspace
 * holds no factors of a converged J) gets NaN gradients, and with gx_mode 1
 * the summed d_gx is NaN.  Errors: PF_E_INVALID (NULL output, bad mode or
 * negative stride, d_gx without d_r and d_x), PF_E_WORKSPACE (ws_stride
 * below ws_doubles; with B > 1 a stride below its row, as
 * pf_adjoint_params).                                                      */
int pf_adjoint(const pf_symbolic sym, int B, double* d_ws, int64_t ws_stride,
               const double* d_gVm, const double* d_gVa, int64_t gv_stride,
               const int8_t* d_type, int64_t type_stride, const double* d_Vm,
               const double* d_Va, int64_t v_stride, const double* d_r, const double* d_x,
               int64_t branch_stride, const int32_t* d_status, double* d_lam,
               int64_t lam_stride, double* d_gP, double* d_gQ, int64_t g_stride, double* d_gx,
               int gx_mode, void* stream);

/* ---- batches of cases with their own sparsity (N-1 outages, mixed grids) --
 * A plan binds G cases to uploaded symbolics (several cases may share one).
 * Per-case arrays are concatenated; pf_multi_info gives each case's element
 * offsets: bus arrays (type, Psp, Qsp, Vm, Va: n of its grid), branch
 * arrays (r, x, b: m of its grid), admittance values (2*nnz_y doubles) and
 * workspace (ws_doubles).  Cases run largest first, one workgroup each, in
 * one launch, unless pf_multi_set_spread gives the launch more workgroups
 * than cases.                                                              */
int pf_multi_create(int G, const pf_symbolic* syms, pf_multi* out);
/* Workgroups of pf_newton_multi's launch (0 or up to G: one per case, the
 * default; at most 65535).  The workgroups beyond one per case go one at a
 * time to the case with the most estimated work per workgroup (a case takes
 * at most one per 128 nodes of its widest level below its LDS tail, and
 * 32), so the largest grids, which bound the launch, share their wide levels
 * among several CUs as a spread one-case launch does (grid barriers within
 * each case's group); below the cut level that info.sub_levels reports,
 * each workgroup of a group takes whole subtrees of the elimination tree
 * (those with their work in its share of the case's) and runs those levels
 * with workgroup barriers only.  The launch is cooperative; when the device cannot
 * keep every workgroup resident at once, or the stream is being captured,
 * it falls back to one workgroup per case.  Changes the plan's device table:
 * pf_multi_info's dev_bytes and pf_multi_upload again before the next call. */
int pf_multi_set_spread(pf_multi plan, int workgroups);
/* offsets: each int64[G+1] (prefix sums), any may be NULL.               */
int pf_multi_info(const pf_multi plan, size_t* dev_bytes, int64_t* bus_off,
                  int64_t* branch_off, int64_t* y_off, int64_t* ws_off);
int pf_multi_upload(pf_multi plan, void* d_buf, size_t bytes, void* stream);
/* d_ysh: bus shunts as (g, b) pairs at twice the bus offsets (16-byte
 * aligned), or NULL for none.                                              */
int pf_build_ybus_multi(const pf_multi plan, const double* d_r, const double* d_x,
                        const double* d_b, const double* d_ysh, double* d_yval, void* stream);
int pf_newton_multi(const pf_multi plan, const double* d_yval, const int8_t* d_type,
                    const double* d_Psp, const double* d_Qsp, double* d_Vm, double* d_Va,
                    double tol, int max_iter, int flags, double* d_ws, int32_t* d_iters,
                    double* d_norm, int32_t* d_status, int32_t* d_pivot, void* stream);
void pf_multi_destroy(pf_multi plan);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
