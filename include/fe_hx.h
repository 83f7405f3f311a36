/*
 * fe_hx.h -- C-ABI of the MI355X (gfx950) matrix-free finite-element
 * Kohn-Sham operator library (libfehx.so).
 *
 * The library applies the FE-discretised Kohn-Sham Hamiltonian to a block of
 * vectors, Y = H X (eqn HX), with
 *     H = T + L + G - i K + sum_a sum_s F_s h_s F_s^*
 * (eqn Hloc: kinetic, local potential, GGA gradient and Bloch-shift terms;
 *  eqn Vnonloc: separable nonlocal projectors), matrix-free on hexahedral
 * spectral cells (Sec. 3.2, eqns ggaReal / ggaCmplx, Alg. 2), and runs the
 * residual Chebyshev filter (Alg. 4) and the Rayleigh-Ritz step (Alg. 3)
 * around it.
 *
 * Conventions shared by every entry point
 *  - Status: every function returns an fe_status; 0 (FE_OK) is success.
 *    Nothing aborts or throws across this boundary; fe_last_error() gives a
 *    thread-local message for the last failure on the calling thread.
 *  - Mesh: a periodic parallelepiped box, lattice rows a_0, a_1, a_2 (bohr,
 *    right-handed), split into ncell[0] x ncell[1] x ncell[2] affine cells;
 *    cell id c = c0 + N0 (c1 + N1 c2).  Reference -> physical map
 *    x = x_c + J (xi + 1), J[:, d] = a_d / (2 N_d)  (Sec. 3.1: one Jacobian
 *    per cell).  Any right-handed parallelepiped (det A > 0; FE_EINVAL
 *    otherwise); a sheared box has an off-diagonal metric J^-1 J^-T, handled
 *    by the kernels.  ncell[d] >= 2 (FE_EUNSUPPORTED otherwise).
 *  - Boundary conditions per axis: periodic[d] != 0 is periodic (Bloch, with
 *    the k-point); periodic[d] == 0 puts homogeneous Dirichlet conditions on
 *    the two faces normal to a_d (non- and semi-periodic systems); the
 *    k-point component along such an axis must be 0 (FE_EINVAL otherwise).
 *  - DoFs: node (i, j, k) of cell c (i along a_0, local I = i + n_p (j + n_p k))
 *    has index h_d = c_d p + i_d along axis d.  Periodic axis: g_d = h_d mod
 *    (N_d p), M_d = N_d p (the wrap is the constraint C of eqn HX).
 *    Dirichlet axis: nodes with h_d = 0 or N_d p carry no DoF (fixed at 0),
 *    the others are g_d = h_d - 1, M_d = N_d p - 1.  DoF id
 *    g_0 + M_0 (g_1 + M_1 g_2); ndofs = M_0 M_1 M_2.
 *  - Quadrature: n_q Gauss-Legendre points per direction (eqn cellIntegrals),
 *    point (q1, q2, q3) of cell c has index c n_q^3 + q1 + n_q (q2 + n_q q3).
 *    n_q = n_p (the reduced rule the filter uses, Sec. 5.3), n_q = n_p + 2
 *    (the accurate default rule, Sec. 5.3) or n_q = n_p + 3 (the rule of the
 *    paper's quadrature-cost remark); n_p = p + 1.  The first two have FP64,
 *    FP32 and BF16 kernels, n_p + 3 FP64 and FP32 ones (BF16 blocks return
 *    FE_EUNSUPPORTED); a vector tile whose LDS block does not fit the device
 *    returns FE_EUNSUPPORTED.
 *  - Multivectors: row-major [ndofs][ld] with the vectors fastest, nvec <= ld,
 *    in device memory owned by the caller.  Element type by precision:
 *        real meshes:    FE_F64 double, FE_F32 float, FE_BF16 bfloat16 bits
 *        complex meshes: FE_F64 complex double (re, im interleaved),
 *                        FE_F32 complex float, FE_BF16 (re, im) bfloat16 pairs
 *    ld and nvec count elements of that type (complex numbers for complex
 *    meshes).  Input and output blocks must not alias.
 *  - Streams: 'stream' is a hipStream_t passed as void* (NULL = null stream).
 *    Work is only enqueued; device faults surface as FE_EDEVICE on a later
 *    call.  A mesh handle may be used by one host thread at a time.
 *  - Host arrays passed in are copied before return; the caller keeps
 *    ownership.  Device buffers the mesh allocates are freed by
 *    fe_mesh_destroy.
 */
#ifndef FE_HX_H
#define FE_HX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fe_mesh_s *fe_mesh_t;
typedef struct fe_filter_graph_s *fe_filter_graph_t;
typedef struct fe_server_s *fe_server_t;
typedef int32_t fe_status;

enum {
  FE_OK = 0,
  FE_EINVAL = -1,        /* NULL pointer, bad size, shape mismatch         */
  FE_ENOMEM = -2,        /* device or host allocation failed               */
  FE_EDEVICE = -3,       /* a HIP / rocBLAS / rocSOLVER call failed        */
  FE_ESTATE = -4,        /* call made in the wrong state                   */
  FE_EUNSUPPORTED = -5   /* valid request this build does not implement    */
};

enum { FE_F64 = 0, FE_F32 = 1, FE_BF16 = 2 };
enum { FE_MASS_LUMPED = 0, FE_MASS_CONSISTENT = 1 };

typedef struct {
  double lattice[3][3];  /* rows: box vectors a_0, a_1, a_2 (bohr)           */
  int32_t ncell[3];      /* cells per axis, >= 2                            */
  int32_t degree;        /* FE degree p = FEOrder, 2 <= p <= 8              */
  int32_t nq;            /* Gauss points per direction: p + 1, p + 3, p + 4 */
  int32_t periodic[3];   /* per axis: 1 periodic, 0 Dirichlet faces         */
  double kpoint[3];      /* Bloch wavevector k (1/bohr)                      */
  int32_t is_complex;    /* 1: complex operator and vectors (forced if k!=0)*/
  int32_t device;        /* HIP device ordinal; -1: host-only mesh (tables, */
                         /* maps, quadrature points, projector assembly;   */
                         /* operator calls return FE_ESTATE)               */
} fe_mesh_desc;

/* One nonlocal projector (eqn Vnonloc).  chi_{lm}(r) = S_lm(r)
 * exp(-|r|^2 / (2 sigma^2)) (1 - |r|^2 / rc^2)^2 for |r| < rc, with the real
 * solid harmonics S indexed m = 0..2l:  l = 0: 1;  l = 1: x, y, z;
 * l = 2: xy, yz, zx, x^2 - y^2, 3 z^2 - r^2.  h is the coupling constant. */
typedef struct {
  int32_t atom;
  int32_t l;
  int32_t m;
  double sigma;
  double rc;
  double h;
} fe_projector;

int32_t fe_abi_version(void);
const char *fe_last_error(void);

/* Build the mesh: host tables (GLL nodes, Gauss rule, 1D shape-function and
 * collocation-derivative matrices), the Jacobian and metric, and the device
 * copies.  *out receives the handle (NULL on failure). */
fe_status fe_mesh_create(const fe_mesh_desc *desc, fe_mesh_t *out);
fe_status fe_mesh_destroy(fe_mesh_t mesh);

/* Sizes: unique DoFs, cells, quadrature points per cell, and the device bytes
 * the mesh currently holds (tables, coefficients, projectors, workspace). */
fe_status fe_mesh_query(fe_mesh_t mesh, int64_t *ndofs, int64_t *ncells,
                        int64_t *nq3, int64_t *footprint_bytes);

/* Cell -> DoF map Q^(e) of eqn HX for cells [first, first + count): host
 * output dofs[(c - first) n_p^3 + I]; -1 for a node on a Dirichlet face.
 * Exact integers, for checking. */
fe_status fe_mesh_cell_dofs(fe_mesh_t mesh, int64_t first, int64_t count,
                            int32_t *dofs);

/* Physical quadrature points of every cell, host output xyz[E n_q^3][3]. */
fe_status fe_mesh_quad_points(fe_mesh_t mesh, double *xyz);

/* The GLL-lumped mass D (diagonal, Sec. 5.3 R-ChFSI), host output [ndofs]. */
fe_status fe_mesh_lumped_mass(fe_mesh_t mesh, double *d);

/* Distorted cells (Sec. 3.1 with a Jacobian per quadrature point): displace
 * the vertices of a periodic box's N0 x N1 x N2 vertex grid by vdisp (host,
 * [N2][N1][N0][3] bohr, vertex (i, j, k) at (i/N0) a_0 + (j/N1) a_1 +
 * (k/N2) a_2 + vdisp[i + N0 (j + N1 k)], copied).  Corner (a, b, c) of cell
 * (c0, c1, c2) is vertex (c0 + a, c1 + b, c2 + c) modulo the grid at its
 * unwrapped lattice position, and each cell is the trilinear image of the
 * reference cube through its eight corners; every integral then takes
 * J(xi_Q), det J(xi_Q) at each quadrature point and the lumped mass det J at
 * each node.  vdisp = NULL restores the affine cells.  The potential returns
 * to zero and the projectors are cleared (set them again).  All three axes
 * must be periodic (FE_EUNSUPPORTED otherwise); a displacement that folds a
 * cell (det J <= 0 at a quadrature point or node) returns FE_EINVAL and
 * leaves the mesh unchanged.  Distorted cells run the general-metric kernels
 * (FP64 and FP32; BF16 blocks take the vector-ALU kernel). */
fe_status fe_mesh_set_geometry(fe_mesh_t mesh, const double *vdisp);

/* Local potential fields at the quadrature points (host, copied):
 * vloc[E n_q^3]  = V_eff (the library adds |k|^2 / 2, eqn Vloc);
 * vgga[E n_q^3][3] = the GGA vector field V^G (eqn den), or NULL for none.
 * The library stores the weighted reference-frame diagonals of eqn refact:
 * (V_eff + |k|^2/2) w det J and sum_a (J^-1)_{s a} V^G_a w det J. */
fe_status fe_set_potential(fe_mesh_t mesh, const double *vloc, const double *vgga);

/* Nonlocal projectors (eqn Vnonloc, eq nlps): natoms positions (host,
 * [natoms][3], bohr, wrapped into the box by the library) and nproj
 * projectors.  Requires rc < half the smallest box width.  The library
 * integrates F_{I,s} = int sum_r exp(-i k.(x - L_r)) chi_s N_I on the cells
 * that meet each projector's support.  nproj = 0 clears the term. */
fe_status fe_set_projectors(fe_mesh_t mesh, int32_t natoms, const double *pos,
                            int32_t nproj, const fe_projector *proj);

/* The assembled projector matrix F of eqn Vnonloc (node rows, projector
 * columns) as host triplets.  Call with rows = cols = vals = NULL to get
 * *nnz, then with arrays of nnz entries (vals: nnz doubles, 2 nnz (re, im)
 * for complex meshes).  Rows ascending, columns ascending within a row. */
fe_status fe_projector_entries(fe_mesh_t mesh, int64_t *nnz, int32_t *rows,
                               int32_t *cols, double *vals);

/* Y = H X for nvec vectors (Alg. 1 on one subdomain with Alg. 2 per cell).
 * The projector reduction F^H X runs before the local-operator launches and
 * the projector update after them.  FE_F64 runs all three on 'stream'; for
 * FE_F32 / FE_BF16 the reduction runs on a second stream the mesh owns,
 * concurrently with the local launches, forked from and joined back into
 * 'stream' with events.  Either way callers see ordinary stream order (and
 * graph capture on 'stream' captures all of it).
 * X, Y: device [ndofs][ldx], [ndofs][ldy] of the precision's element type.
 * FE_F64 is the reference path; FE_F32 computes in float; FE_BF16 reads and
 * writes bfloat16 and computes in float.  Enqueued on 'stream'. */
fe_status fe_apply_H(fe_mesh_t mesh, const void *X, int64_t ldx, void *Y,
                     int64_t ldy, int64_t nvec, int32_t prec, void *stream);

/* fe_apply_H for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same Y = H X with the same kernels, arguments, layout and errors as
 * fe_apply_H, but it calls no hipMalloc / hipFree / hipStreamCreate and no
 * allocating library routine.  The projector term's per-chunk partials and W
 * live in one static device array of FE_NOALLOC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends; a call
 * whose projector workspace ((chunks x 10 + projectors) x ceil4(real lanes)
 * x 8 bytes) exceeds it returns FE_EINVAL.  The projector reduction runs on
 * 'stream' itself in every precision.  All calls on one device
 * share that array: calls that overlap on one device (two streams, or two
 * host threads) race and must be serialised by the caller.  Nothing in it
 * needs to start at zero; each call writes the partials and W before it
 * reads them. */
#define FE_NOALLOC_SCRATCH_BYTES (32LL << 20)
fe_status fe_apply_H_noalloc(fe_mesh_t mesh, const void *X, int64_t ldx, void *Y,
                             int64_t ldy, int64_t nvec, int32_t prec, void *stream);

/* Y = M X with the consistent FE mass matrix M = sum_e Q^T N3^T (w det J) N3 Q
 * (eqn FEeigen's overlap matrix, Gauss quadrature of the mesh), matrix-free
 * on the same kernel as fe_apply_H.  Blocks and precisions as fe_apply_H. */
fe_status fe_apply_M(fe_mesh_t mesh, const void *X, int64_t ldx, void *Y,
                     int64_t ldy, int64_t nvec, int32_t prec, void *stream);

/* Which mass matrix the eigensolver entry points use for H u = eps M u:
 * FE_MASS_LUMPED (default): M = D, the GLL-lumped diagonal;
 * FE_MASS_CONSISTENT: the residual Y = H X - M X Lambda of fe_cheb_filter and
 * the Gram matrix Y^H M Y of fe_rayleigh_ritz use the consistent M (applied
 * matrix-free in FP64); the filter's approximate inverse stays D^-1 (Alg. 4)
 * and fe_lanczos still bounds D^-1/2 H D^-1/2. */
fe_status fe_set_mass(fe_mesh_t mesh, int32_t kind);

/* Residual Chebyshev filter of Alg. 4 (M = D, or the consistent M after
 * fe_set_mass(FE_MASS_CONSISTENT); D^-1 is always the lumped inverse):
 * X (device, FP64 element type, [ndofs][ldx]) holds X^(i) on entry and the
 * filtered block on return; lam (device, double[nvec]) holds Lambda^(i).
 * The residual Y = H X - D X Lambda, X Lambda_Y and the final combine run
 * in FP64; the degree-1 recurrence steps (H D^-1 - c) R_Y run in
 * inner_prec (FE_F64, FE_F32 or FE_BF16 storage/compute as in fe_apply_H).
 * The library keeps a workspace of 3-4 blocks of nvec vectors on the mesh
 * (counted in the footprint; allocated on first use, which synchronises):
 * FP64 inner steps 4 x 8 bytes per element, FP32 16 bytes and BF16 12
 * bytes (the FP64 residual shares the R_X block).
 * Otherwise only enqueued on 'stream': no host synchronisation, lam is read
 * on the device.  One pass per mesh may be in flight at a time. */
fe_status fe_cheb_filter(fe_mesh_t mesh, void *X, int64_t ldx, const double *lam,
                         int64_t nvec, int32_t degree, double lam_min,
                         double lam_T, double lam_max, int32_t inner_prec,
                         void *stream);

/* One fe_cheb_filter pass captured once as a HIP graph and replayed: the
 * graph holds every launch of the pass (Lambda tables from the device Ritz
 * values, the FP64 residual, the degree-1 recurrence steps, the final
 * combine) for the given X, lam, nvec, degree, bounds and inner precision;
 * each launch reads the current contents of X and lam.  Create allocates the
 * mesh's filter workspaces; launch only enqueues (no host synchronisation);
 * results equal fe_cheb_filter's bit for bit.  The graph uses the mesh's
 * workspaces: no other filter, Rayleigh-Ritz or Lanczos call on the same mesh
 * may overlap a launch.  While a graph is alive the mesh never frees or moves
 * the buffers it holds: a call that would need a larger filter or projector
 * workspace (fe_cheb_filter with more vectors or another inner precision's
 * layout, fe_apply_H with more vectors) or new projector data
 * (fe_set_projectors) returns FE_ESTATE instead, and so does fe_mesh_destroy.
 * Destroy the graph first. */
fe_status fe_filter_graph_create(fe_mesh_t mesh, void *X, int64_t ldx, const double *lam,
                                 int64_t nvec, int32_t degree, double lam_min,
                                 double lam_T, double lam_max, int32_t inner_prec,
                                 fe_filter_graph_t *graph);
fe_status fe_filter_graph_launch(fe_filter_graph_t graph, void *stream);
fe_status fe_filter_graph_destroy(fe_filter_graph_t graph);

/* Lanczos on D^-1/2 H D^-1/2 in FP64 with full reorthogonalisation (the
 * spectral-bound estimate Alg. 4 takes as input): 'steps' iterations from
 * the device start vector v0 [ndofs] (FP64 element type).  Host outputs:
 * theta[steps] (Ritz values, ascending) and *beta_last.  Synchronous. */
fe_status fe_lanczos(fe_mesh_t mesh, const void *v0, int32_t steps,
                     double *theta, double *beta_last);

/* Rayleigh-Ritz step of Alg. 3 with M = D (or the consistent M, see
 * fe_set_mass), in FP64 (rocBLAS gemm,
 * rocSOLVER Cholesky and symmetric/Hermitian eigensolver):
 * (Y^H H Y) E = (Y^H D Y) E Lambda, then X = Y E in place.
 * X: device FP64 block [ndofs][ldx]; ritz: device double[nvec] output,
 * ascending.  Synchronous.  FE_EDEVICE when Y^H D Y is not positive
 * definite (Y rank-deficient) or the eigensolver does not converge; X is
 * then left unspecified. */
fe_status fe_rayleigh_ritz(fe_mesh_t mesh, void *X, int64_t ldx, int64_t nvec,
                           double *ritz, void *stream);

/* Y_i = H_i X_i for n systems (meshes on one device) in as few launches as
 * possible: the local operator of all systems of one class (degree,
 * quadrature, real/complex, vector tile) runs as one persistent launch per
 * colour phase over the concatenated (column, vector tile) work lists of up
 * to 8 systems at a time; the nonlocal terms follow per system.  Arrays of n
 * entries (host): meshes, X[i] / Y[i] device blocks as in fe_apply_H with
 * ldx[i], ldy[i], nvec[i]; each mesh at most once per call.  Results equal n
 * separate fe_apply_H calls bit for bit.  Enqueued on 'stream'. */
fe_status fe_batch_apply(int32_t n, const fe_mesh_t *meshes, const void *const *X,
                         const int64_t *ldx, void *const *Y, const int64_t *ldy,
                         const int64_t *nvec, int32_t prec, void *stream);

/* Launch-shape tuning of the local operator.  kind 0: plain H X (fe_apply_H,
 * Rayleigh-Ritz, the filter's residual); kind 1: filter steps
 * (fe_cheb_filter: H D^-1 R, D^-1 applied while gathering).  vt is the vector tile in real lanes per workgroup:
 * {2, 4, 8, 16} for FE_F64, plus 10 where n_q = n_p (2 only where 4 does not
 * fit the LDS), {8, 16, 32} for FE_F32 / FE_BF16 (the matrix-core BF16 kernel
 * runs 8 as 16); 0 restores the built-in default.  fe_set_tile refuses
 * (FE_EINVAL) a tile whose local-operator block does not fit the LDS on this
 * mesh (16 FP64 lanes at n_p = 8, two lanes wherever four fit, ...).
 * fe_autotune runs every
 * candidate tile 'reps' times on scratch blocks of nvec vectors (allocated and
 * freed inside; synchronous), keeps the fastest on the mesh and returns it;
 * cand_vt / cand_ms (host, FE_TILE_CANDIDATES entries, may be NULL) receive
 * each candidate's time per application in ms (-1: does not fit), *ncand
 * their count. */
#define FE_TILE_CANDIDATES 8
fe_status fe_set_tile(fe_mesh_t mesh, int32_t prec, int32_t kind, int32_t vt);
fe_status fe_get_tile(fe_mesh_t mesh, int32_t prec, int32_t kind, int32_t *vt);
fe_status fe_autotune(fe_mesh_t mesh, int32_t prec, int32_t kind, int64_t nvec,
                      int32_t reps, int32_t *best_vt, int32_t *cand_vt,
                      double *cand_ms, int32_t *ncand);

/* The eigensolver loop of Alg. 3 with the Alg. 4 filter and M = D:
 *   Lanczos (lanczos_steps, from v0)  ->  lam_max = largest Ritz value +
 *   |last beta|;  Rayleigh-Ritz of the starting block X;  then 'outer' passes
 *   of  filter(degree, inner_prec) + Rayleigh-Ritz.
 * Bounds per pass (the paper leaves them to the caller): pass 1 takes
 * lam_min = smallest Lanczos Ritz value and lam_T = lam_min + the
 * free-electron energy below which the box holds nvec states,
 * (1/2)(6 pi^2 nvec / volume)^(2/3); later passes take the smallest and the
 * largest Ritz value of the previous Rayleigh-Ritz step.
 * X: device FP64 block [ndofs][ldx], replaced by the Ritz vectors; v0:
 * device FP64 element type [ndofs]; ritz: HOST double[nvec] output
 * (ascending); bounds: NULL or HOST double[3 outer] receiving (lam_min,
 * lam_T, lam_max) of every pass.  Uses the filter / Lanczos / Rayleigh-Ritz
 * workspaces and one more of nvec doubles.  Synchronous. */
fe_status fe_chfsi(fe_mesh_t mesh, void *X, int64_t ldx, int64_t nvec,
                   const void *v0, int32_t outer, int32_t degree,
                   int32_t lanczos_steps, int32_t inner_prec, double *ritz,
                   double *bounds, void *stream);

/* ---- request server (continuous batching over resident meshes) ----------
 * A request names a resident mesh and a caller-owned device block:
 *   FE_REQ_APPLY   Y = H X (prec: element type of X and Y, as fe_apply_H);
 *   FE_REQ_FILTER  one fe_cheb_filter pass on X in place (X FP64; prec: the
 *                  inner precision; lam device Ritz values; degree, bounds).
 * The server runs on one device and one stream.  Each tick it retires
 * finished requests, admits queued ones (FIFO, first fit) while fewer than
 * max_active run, the request's mesh is idle and the device bytes held by
 * the meshes it has served plus the request's new workspace stay within
 * hbm_budget (idle meshes' request workspaces are released to make room),
 * and advances every active request by one filter step, with the local
 * operators of all active requests of one launch class in one persistent
 * batched launch (fe_batch_apply's kernel).  Results are identical to running
 * each request alone.  The caller keeps X, Y, lam and the mesh alive and
 * unchanged until the request is done, must not use a mesh with a queued
 * or active request elsewhere, and must keep every mesh it submitted for
 * alive until fe_server_destroy (the server counts their device bytes).  Timestamps are host steady-clock seconds:
 * submit, admission, completion (when progress observed it). */
enum { FE_REQ_APPLY = 0, FE_REQ_FILTER = 1 };
typedef struct {
  fe_mesh_t mesh;
  int32_t kind;
  int32_t prec;
  void *X;
  int64_t ldx;
  int64_t nvec;
  void *Y;             /* FE_REQ_APPLY only */
  int64_t ldy;
  const double *lam;   /* FE_REQ_FILTER only: device [nvec] */
  int32_t degree;
  double lam_min, lam_T, lam_max;
} fe_request;

fe_status fe_server_create(int32_t device, int64_t hbm_budget, int32_t max_active,
                           fe_server_t *server);
/* Queue a request (copied); FE_ENOMEM if it can never fit the budget. */
fe_status fe_server_submit(fe_server_t server, const fe_request *req, int64_t *id);
/* One scheduler round.  block = 0: never waits (at most two ticks are kept
 * in flight); block = 1: waits for the oldest tick or a completion when it
 * cannot enqueue more.  Returns the active and queued counts. */
fe_status fe_server_progress(fe_server_t server, int32_t block, int32_t *n_active,
                             int32_t *n_queued);
/* Progress until every request is done or failed. */
fe_status fe_server_drain(fe_server_t server);
/* state: 0 queued, 1 active, 2 done, 3 failed (err = its status);
 * times[3] = submit, admission, completion. */
fe_status fe_server_status(fe_server_t server, int64_t id, int32_t *state, double *times,
                           int32_t *err);
fe_status fe_server_stats(fe_server_t server, int64_t *ticks, int64_t *held_bytes);
/* Request workspaces: when a request completes, its mesh's filter blocks and
 * projector reduction block return to the server's pool of idle buffers, and
 * an admission takes the smallest idle buffer per slot that holds it (at most
 * four times its size) before it allocates; the pool's bytes count against the
 * budget and are freed, largest first, only when an admission needs room.
 * allocs / frees: device allocations and frees the server has made for
 * request workspaces; idle_bytes: the pool's current bytes.  Any output may be
 * NULL. */
fe_status fe_server_pool_stats(fe_server_t server, int64_t *allocs, int64_t *frees,
                               int64_t *idle_bytes);
/* Admission work cap: with cap > 0 no request joins a non-empty batch that
 * would then apply H to more than 'cap' DoF x real lanes per step in total
 * (DoFs x nvec, x2 for complex meshes); the queue then waits in arrival
 * order.  A request that fills the device on its own runs alone, small ones
 * share steps.  0 (the default) admits up to max_active requests. */
fe_status fe_server_set_work_cap(fe_server_t server, int64_t cap);
/* Waits for the server's stream, then frees the server (not the meshes). */
fe_status fe_server_destroy(fe_server_t server);

#ifdef __cplusplus
}
#endif
#endif /* FE_HX_H */
