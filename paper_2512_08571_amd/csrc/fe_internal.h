// Internal declarations of libfehx (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fe_hx.h"

namespace fehx {

// ---- error reporting ------------------------------------------------------
fe_status set_error(fe_status code, const std::string &msg);
#define FE_HIP_TRY(expr)                                                       \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess)                                                      \
      return ::fehx::set_error(FE_EDEVICE, std::string(#expr) + ": " +         \
                                               hipGetErrorString(_e));         \
  } while (0)

// Coefficient blocks per cell and quadrature point on the general-metric
// path (sheared boxes, distorted cells), all weighted by w_Q det J(xi_Q):
//   0: V_eff + |k|^2/2;  1-3: sum_a (J^-1)_{s a} V^G_a;
//   4-6: (1/2)(J^-1 J^-T)_{ss};  7-9: (1/2)(J^-1 J^-T)_{01, 02, 12};
//   10-12: sum_a (J^-1)_{s a} k_a.
// Plain meshes keep only blocks 0-3 (the metric is in the 1D tables).
constexpr int NCOEF_GEN = 13;
// LDS bytes of one staged local-operator block (the kernels' lds_need):
// two [n_q^3][vt] buffers, two carried planes, the coefficient blocks, the
// line weights, and with the general metric three staged gradients
constexpr size_t LOCAL_LDS_MAX = 160 * 1024;
constexpr size_t local_lds_bytes(int np, int nq, int vt, int bytes, bool offd) {
  return ((size_t)(2 * nq * nq * nq + 2 * np * np) * vt + (size_t)(offd ? NCOEF_GEN : 4) * nq * nq * nq + nq * nq +
          (offd ? (size_t)3 * nq * nq * nq * vt : 0)) * bytes;
}

// support nodes per chunk of the nonlocal W = F^H X reduction
constexpr int NL_CHUNK = 1024;
constexpr int NL_MAXP = 10;     // projectors per atom the nonlocal kernels handle (s, p, d = 9)
constexpr int NL_BPMAX = 64;    // projectors whose W rows one brick of the update stages in LDS

// ---- 1D tables (Sec. 2.2 GLL basis, eqn cellIntegrals Gauss rule) ---------
struct Tables1D {
  int p = 0, np = 0, nq = 0;
  std::vector<double> gll, gllw;   // GLL nodes / weights (np)
  std::vector<double> xq, wq;      // Gauss points / weights (nq)
  std::vector<double> N;           // N[q*np + i]  = l_i(xq_q)
  std::vector<double> Dt;          // Dt[q*nq + r] = d/dxi of the Gauss-point
                                   // Lagrange polynomial r at xq_q (collocation)
};
Tables1D make_tables(int p, int nq);

// Even-odd packing of a centro-(anti)symmetric matrix A[nout][nin]: rows
// q < ceil(nout/2): E[q][0..ceil(nin/2)) then O[q][0..floor(nin/2)).
std::vector<double> eo_pack(const std::vector<double> &A, int nout, int nin, int sym);

// offsets (in elements) inside one table buffer: the four packed matrices,
// then per direction D the point factors g_DD w_i det J and kappa_D w_i det J
// (w_i the 1D Gauss weights), [3][nq] each
struct TabLayout {
  int n_off, nt_off, d_off, dt_off, gw_off, kw_off, total;
};
inline TabLayout tab_layout(int np, int nq) {
  TabLayout t;
  t.n_off = 0;
  t.nt_off = t.n_off + ((nq + 1) / 2) * np;
  t.d_off = t.nt_off + ((np + 1) / 2) * nq;
  t.dt_off = t.d_off + ((nq + 1) / 2) * nq;
  t.gw_off = t.dt_off + ((nq + 1) / 2) * nq;
  t.kw_off = t.gw_off + 3 * nq;
  t.total = t.kw_off + 3 * nq;
  return t;
}

// ---- local-operator launch description --------------------------------------
struct LocalLaunch {
  const void *X = nullptr;
  void *Y = nullptr;
  int64_t ldx = 0, ldy = 0;   // in real lanes
  int nlanes = 0;             // real lanes (complex: 2 nvec)
  int prec = FE_F64;
  const double *dinv_gather = nullptr;  // scale gathered X by D^-1 (filter)
  bool mass = false;          // the consistent mass operator M instead of H
  int vt = 0, nt = 0;         // vector tile / threads (0: tuned default)
  bool store32 = false;       // FE_BF16 arithmetic on FP32 blocks (the filter's recurrence state)
};

struct Mesh;
// Several local-operator applications of one class (degree, quadrature,
// real/complex, precision, vector tile) launched together.
struct LocalBatch {
  Mesh *const *ms = nullptr;
  const LocalLaunch *Ls = nullptr;
  int n = 0;
  bool persistent = false;   // use the persistent batched kernel even for n = 1
  int blocks_per_cu = 0;     // persistent grid per CU (0: occupancy limit)
};
fe_status launch_local(Mesh *m, const LocalLaunch &L, hipStream_t s);
fe_status launch_local_batch(const LocalBatch &B, hipStream_t s);
fe_status ensure_nl_workspace(Mesh *m, int nlanes);
int64_t nl_workspace_bytes(const Mesh *m, int nlanes);
fe_status launch_nonlocal_w(Mesh *m, const void *X, int64_t ldx, int nlanes, int prec, const double *dinv,
                            hipStream_t s);
fe_status launch_nonlocal_y(Mesh *m, void *Y, int64_t ldy, int nlanes, int prec, double alpha, hipStream_t s);
fe_status ensure_side_stream(Mesh *m);
// projector reduction before the local launches (FP32 / BF16: forked to the
// mesh's second stream) and the update after them (joining that stream)
fe_status nonlocal_reduce(Mesh *m, const void *X, int64_t ldx, int nlanes, int prec, const double *dinv,
                          hipStream_t s);
fe_status nonlocal_update(Mesh *m, void *Y, int64_t ldy, int nlanes, int prec, double alpha, hipStream_t s);
fe_status apply_with_nonlocal(Mesh *m, const LocalLaunch &L, int prec, const double *dinv, double alpha,
                              hipStream_t s);

// One residual Chebyshev filter pass (Alg. 4, M = D) broken into the pieces
// an eager call, a captured graph and the step-batching server enqueue:
// setup (host scalars, workspaces; may allocate), prologue, per-step local
// launch description + nonlocal part, final combine.  Only setup allocates or
// synchronises; everything else only enqueues.  The plan uses the mesh's
// filter workspaces, so one pass per mesh may be in flight at a time.
struct FilterPlan {
  Mesh *m = nullptr;
  double *X = nullptr;
  int64_t ldx = 0;                 // real lanes
  const double *lam = nullptr;     // device [nvec]
  int64_t nvec = 0;
  int lanes = 0, degree = 0, prec = 0;
  int sprec = 0;                   // element type of the recurrence blocks: FE_F64, or FE_F32 (FP32 and BF16 steps)
  double e = 0, c = 0, sigma1 = 0;
  std::vector<double> alpha, s2;   // per step k = 2..degree: 2 sigma2 / e, sigma sigma2
  double *Y = nullptr, *tab = nullptr;
  void *RY = nullptr, *RX = nullptr, *Ylp = nullptr, *T = nullptr;
  int k = 2;                       // next recurrence step
};
fe_status filter_setup(FilterPlan &P, Mesh *m, double *X, int64_t ldx_lanes, const double *lam, int64_t nvec,
                       int degree, double lmin, double lT, double lmax, int prec);
fe_status filter_prologue(FilterPlan &P, hipStream_t s);
LocalLaunch filter_step_local(const FilterPlan &P);
fe_status filter_step_reduce(FilterPlan &P, hipStream_t s); // projector reduction of step P.k
fe_status filter_step_rest(FilterPlan &P, hipStream_t s);   // projector update of step P.k, then advance
fe_status filter_final(FilterPlan &P, hipStream_t s);
fe_status launch_nonlocal(Mesh *m, const void *X, int64_t ldx, void *Y, int64_t ldy,
                          int nlanes, int prec, const double *dinv_gather,
                          double alpha, hipStream_t s);

// ---- the mesh object ----------------------------------------------------------
struct Mesh {
  fe_mesh_desc desc{};
  int p = 0, np = 0, nq = 0, N[3] = {0, 0, 0}, Mn[3] = {0, 0, 0};
  int64_t E = 0, m = 0;
  bool cplx = false;
  int device = 0;
  bool host_only = false;   // device < 0: host tables and maps only
  double J[3][3]{}, Jinv[3][3]{}, detJ = 0;
  double gdiag[3]{}, kap[3]{}, k2half = 0;
  bool offd = false;          // general-metric kernels: off-diagonal J^-1 J^-T (sheared box) or distorted cells
  bool offd_affine = false;   // the affine map's metric has off-diagonal entries
  bool distorted = false;     // cells are trilinear images of displaced vertices (a Jacobian per point)
  std::vector<double> vdisp;  // host vertex displacements [N0 N1 N2][3] of a distorted mesh
  int ncoef = 4;              // coefficient blocks per cell: 4, or NCOEF_GEN with the per-point metric
  int64_t coefM_cell = 0;     // mass-operator coefficient elements per cell (0: one block for all cells)
  Tables1D t1;

  // device tables / coefficients (compute precision copies)
  double *tab64 = nullptr;
  float *tab32 = nullptr;
  float *tabmx = nullptr;               // [4][8][8] full N, N^T, Dtilde, Dtilde^T (MFMA operands), zero padded
  double *wq64 = nullptr;               // [nq2] w_a w_b: the two 1D weights off a line
  float *wq32 = nullptr;
  // the consistent mass operator on the same kernel: tables without the
  // kinetic and Bloch factors, one coefficient block for every cell
  // ([4][nq3]: w det J, then zeros)
  double *tabM64 = nullptr, *coefM64 = nullptr;
  float *tabM32 = nullptr, *coefM32 = nullptr;
  int mass_kind = 0;                    // filter / Rayleigh-Ritz mass: 0 lumped D, 1 consistent M
  double *coef64 = nullptr;   // [E][4][nq^3]: (V + |k|^2/2) w detJ, then Vtilde_s w detJ
  float *coef32 = nullptr;
  bool has_gga = false;
  double *dmass = nullptr, *dinv = nullptr;   // lumped mass and its inverse [m]
  std::vector<double> h_dmass;

  // column colouring (phases of the deterministic scatter)
  int ncolx = 0, ncoly = 0, nphase = 0;
  int vt_pref[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // vector tile per [precision][epilogue] (0: default)
  hipStream_t side = nullptr;                       // FP32 / BF16 projector reduction beside the local launches
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int *cols = nullptr;        // device int2 list, phases concatenated
  std::vector<int> phase_off; // nphase + 1

  // nonlocal
  int natoms = 0, ns = 0;
  std::vector<double> h_h;              // couplings per projector
  // per-atom dense blocks for W = P^H X
  int *nl_atom_off = nullptr;           // [natoms+1] offsets into support list
  int *nl_atom_nodes = nullptr;         // support nodes, atom-major
  int *nl_atom_proj = nullptr;          // [natoms+1] projector offsets
  double *nl_F64 = nullptr;             // per support node: nproj_a values (x2 if complex)
  float *nl_F32 = nullptr;
  int64_t nl_nsup = 0;
  int nl_maxproj = 0;
  int nl_nchunks = 0;
  int *nl_chunk_atom = nullptr;         // atom of each node chunk
  int *nl_chunk_n0 = nullptr;           // first support-list entry of each chunk
  int *nl_chunk_order = nullptr;        // execution order of the chunks (by position)
  int *nl_atom_chunk0 = nullptr;        // [natoms+1] chunk offsets
  int *nl_proj_atom = nullptr;          // atom of each projector
  std::vector<int> h_atom_off, h_atom_proj;
  std::vector<int> h_rows, h_rowptr{0}, h_colidx;   // host copy of the node-CSR of P
  std::vector<double> h_val;
  // node-CSR of P for Y += P (h W)
  int *nl_rows = nullptr;               // support rows (node ids)
  int *nl_rowptr = nullptr;             // [nrows+1]
  int *nl_colidx = nullptr;             // projector index
  double *nl_val64 = nullptr;           // value (x2 if complex)
  float *nl_val32 = nullptr;
  int64_t nl_nrows = 0, nl_nnz = 0;     // rows / entries left to the global-W update
  // brick-ordered update rows: brick b owns rows [b_row0[b], b_row0[b+1]) and
  // the projectors b_proj[b_p0[b] ..); a row's entries are groups of four
  // [b_rowptr[r], b_rowptr[r+1]) (zero-padded to an even group count),
  // columns local to the brick's projector list, values [group][4][re, im]
  // (FP32; the FP64 update reads the dense blocks below)
  int nl_nbrick = 0, nl_bmaxp = 0;
  int *nl_b_row0 = nullptr, *nl_b_p0 = nullptr, *nl_b_proj = nullptr;
  int *nl_b_rows = nullptr, *nl_b_rowptr = nullptr;
  int *nl_b_lcol = nullptr;
  float *nl_b_val32 = nullptr;
  // dense FP64 projector block of brick b: rows x nl_b_k[b] values from
  // nl_b_aoff[b], row-major, column C p + c for the brick's projector p and
  // part c (re, im), zero-padded to a multiple of 4 columns
  double *nl_b_A64 = nullptr;
  int64_t *nl_b_aoff = nullptr;
  int *nl_b_k = nullptr;
  int nl_b_kmax = 0;
  double *nl_h = nullptr;               // couplings on device
  void *nl_W = nullptr;                 // workspace ns x lanes (double)
  int64_t nl_W_lanes = 0;

  // filter workspace
  // workspaces: 0 filter Y (FP64), 1 R_Y, 2 R_X, 3 Y in the inner precision,
  // 4 Lambda tables, 5-6 Lanczos / Rayleigh-Ritz, 7 Ritz values, 8 filter H D^-1 R_Y
  // 9 M X (FP64, consistent-mass filter), 10 Rayleigh-Ritz partial Gram matrices.
  // FP32 / BF16 filter: no slots 0 and 8; slot 2 holds R_X and, at
  // filter_t_offset, H D^-1 R_Y, and the FP64 Y (read only by the prologue)
  // spans both (slot 2 padded to 8 bytes per element where they are smaller).
  static constexpr int NWS = 11;
  void *ws[NWS] = {};
  int64_t ws_bytes[NWS] = {};

  int64_t footprint = 0;
  std::vector<std::pair<void *, size_t>> owned;
  // captured filter graphs alive on this mesh: they hold the addresses of the
  // filter and projector workspaces and of the projector arrays, so while
  // any is alive those buffers are never freed or moved (calls that would
  // have to return FE_ESTATE)
  int graphs = 0;

  fe_status dev_alloc(void **p, size_t bytes);
  void dev_free_all();
};

fe_status ensure_workspace(Mesh *m, int slot, int64_t bytes);

// Whether two [rows][ld] blocks of nvec used elements (element size es)
// share an element: X and Y of an application must not.  Blocks whose byte
// ranges interleave with one leading dimension (disjoint column windows of
// one array) do not share one; other overlapping ranges count as sharing.
inline bool blocks_overlap(const void *X, int64_t ldx, const void *Y, int64_t ldy, int64_t rows, int64_t nvec,
                           int64_t es) {
  if (rows <= 0 || nvec <= 0) return false;
  const intptr_t x0 = (intptr_t)X, y0 = (intptr_t)Y;
  const intptr_t x1 = x0 + (intptr_t)(((rows - 1) * ldx + nvec) * es);
  const intptr_t y1 = y0 + (intptr_t)(((rows - 1) * ldy + nvec) * es);
  if (!(x0 < y1 && y0 < x1)) return false;
  if (ldx != ldy || (y0 - x0) % es != 0) return true;
  int64_t c = ((y0 - x0) / es) % ldx;                 // column offset of Y's window in X's rows
  if (c < 0) c += ldx;
  return c < nvec || c > ldx - nvec;
}
// element bytes of a vector block of precision prec (complex meshes: pairs)
inline int64_t block_elem_bytes(int prec, bool cplx) {
  return (prec == FE_F64 ? 8 : (prec == FE_F32 ? 4 : 2)) * (cplx ? 2 : 1);
}

// FP32 / BF16 filter layout (ts = 4 or 2 bytes per element, n = rows x
// lanes elements): H D^-1 R_Y sits in slot 2 after R_X at a 256-byte aligned
// offset, and slot 2 is large enough for the 8 n bytes of the FP64 Y too.
inline int64_t filter_t_offset(int64_t n, int64_t ts) { return (n * ts + 255) / 256 * 256; }
inline int64_t filter_shared_bytes(int64_t n, int64_t ts) {
  const int64_t b = filter_t_offset(n, ts) + n * ts;
  return b > 8 * n ? b : 8 * n;
}

}  // namespace fehx

struct fe_mesh_s : public fehx::Mesh {};
