// C ABI of the Chebyshev-filter library: validation, device data layout,
// colouring, Schur-complement setup and the drivers of the hot path
// (H X, M X, (M^E)^-1 X, the Chebyshev filter, Cholesky-QR, Rayleigh-Ritz,
// Lanczos bounds).  Every arithmetic step runs in the kernels of cf_ops.hip
// and cf_dense.hip; the small dense generalized eigenproblem of the
// Rayleigh-Ritz step is solved on the device by rocSOLVER (dsygvd).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "chebfilter.h"
#include "cf_kernels.h"

using namespace cf;

// cf_mlp.hip
cf_status cf_mlp_predict_raw(cf_mlp *m, const double *x_raw, double *y_raw);
int cf_mlp_n_in(const cf_mlp *m);
int cf_mlp_n_out(const cf_mlp *m);
const char *cf_mlp_err(const cf_mlp *m);

namespace {

struct ProfEntry {
  int64_t launches = 0;
  double ms = 0.0;
  double flops = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

thread_local std::string g_init_error;

}  // namespace

struct cf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int p = 0, npc = 0;
  int64_t E = 0, n_h = 0, n_e = 0, n = 0, max_cols = 0;
  // columns of the column chunk: blocks wider than this are processed chunk
  // by chunk
  int64_t chunk = 0;
  // leading dimension of the internal work blocks: the chunk rounded up to a
  // multiple of 16 doubles, so that every row segment a kernel gathers starts
  // on a 128-byte boundary
  int64_t ldw = 0;
  int check_finite = 0;
  // classical cells
  double *Hp = nullptr;
  int32_t *dofp = nullptr;
  uint8_t *flagp = nullptr;                 // CELL_FIRST / CELL_FINISH per (cell, local node)
  int32_t *regrows = nullptr;               // classical DOFs inside enriched cells
  int64_t nregrows = 0;
  double *dvec = nullptr, *dinv = nullptr;
  int32_t *cells = nullptr;
  std::vector<int> col_off;
  // enrichment: per-cell blocks (transposed, for the partial products), the
  // node-major assembled coupling (CSR over classical DOFs) and dense blocks
  int64_t nnz = 0;
  int kmax = 0;
  double *HT = nullptr, *MT = nullptr;
  int64_t *toff = nullptr;
  int32_t *tld = nullptr;
  int64_t *eptr = nullptr;
  int32_t *ecells = nullptr;
  // the same cells, most enrichment functions first: the coupling-partials
  // launches take them in this order, so the longest workgroups start first
  // (their output rows do not depend on the order)
  int32_t *ecells_part = nullptr;
  // work items of the FP64 coupling partials: (position in ecells_part) * 32
  // + row-block group, laid out so that a cell's groups share an XCD; -1 pads
  int32_t *epitems = nullptr;
  int nepitems = 0;
  int32_t *epos_part = nullptr;             // positions in ecells of the cells of ecells_part
  int necells = 0;
  int64_t *aptr = nullptr;
  int32_t *alist = nullptr;
  double *Hec = nullptr, *Mec = nullptr;   // per-cell blocks, rows padded to NPAD
  int32_t *eidx = nullptr;
  int32_t *qptr = nullptr, *qidx = nullptr; // classical DOF -> rows of the cell buffer Q
  int qmax = 0;                             // most cell-buffer rows of one DOF
  double *Q = nullptr;                      // [necells * NPAD][ldw]
  int64_t csr_nnz = 0, nreg = 0;
  double *Hee = nullptr, *Mee = nullptr, *Sinv = nullptr, *Hmod = nullptr;
  // block workspace, leading dimension ldw
  double *R = nullptr, *P = nullptr, *Wb = nullptr, *Zb = nullptr, *B2 = nullptr, *T = nullptr,
         *U = nullptr;
  // small dense workspace
  double *G = nullptr, *Gp = nullptr, *Wm = nullptr, *Wt = nullptr, *sv = nullptr, *Hh = nullptr,
         *Mh = nullptr, *theta = nullptr, *evE = nullptr;
  int gp_chunks = 8;
  int *flag = nullptr;
  rocblas_int *info = nullptr;
  // Lanczos
  double *lzv = nullptr, *lzcoef = nullptr, *lzpart = nullptr;
  // reduced-precision filter state, allocated on the first CF_FP32 / CF_BF16
  // filter call: FP32 (or BF16) copies of the cell matrices, FP32 copies of
  // the coupling blocks and FP32 recurrence blocks (ld = ldw)
  int64_t ttot = 0;
  float *Hp32 = nullptr;
  void *Hp16 = nullptr;
  float *HT32 = nullptr, *MT32 = nullptr, *Hec32 = nullptr, *Mec32 = nullptr;
  float *F0 = nullptr, *F1 = nullptr, *R32 = nullptr, *P32 = nullptr, *Q32 = nullptr;
  // step scaling of the reduced recurrence: max slots, exponents, multipliers
  unsigned *lp_mx = nullptr;
  int32_t *lp_s = nullptr;
  float *lp_mult = nullptr;
  int lp_cap = 0;
  // cells of each colour reordered: those sharing a DOF with an enriched cell
  // first (near_cnt[k] of them), then the rest; the BF16 form keeps the near
  // ones in FP32
  int32_t *cells_split = nullptr;
  std::vector<int> near_cnt;
  // 16-column MFMA blocks per column tile of the reduced cell product, for
  // the FP32-input cells [0] and the BF16-input cells [1] (chebfilter_autotune)
  int lp_nsb[2] = {1, 2};
  // row-block bucket -> k split of the FP32 coupling partials (2 bits per
  // bucket of 1, 2, 3, >= 4 row blocks; chebfilter_autotune)
  int lp_bmap = CPL_BMAP_DEFAULT;
  // assembly of the plain cells' blocks: reference tables (shape values
  // [nq4][NPAD], weights [nq], kinetic block [NPAD][NPAD]), the uploaded cell
  // list and its host copy, which cells carry enrichment functions
  double *asm_B = nullptr, *asm_w = nullptr, *asm_K = nullptr;
  int asm_nq = 0;
  int32_t *asm_cells = nullptr;
  int64_t asm_cap = 0;
  std::vector<int32_t> asm_list;
  std::vector<uint8_t> cell_enriched;
  // assembly of the cells with their own adaptive rule (chebfilter_enriched_tables):
  // device copies of the listed cells, their leaf boxes, the shared table and
  // the atom centres; the enrichment-row work items and the atom-pair lists
  // of the partial H^ee sums, both grouped in batches whose partial blocks fit
  // the partial buffer (host: the batches' first item and pair)
  struct {
    int ncl = 0, np1 = 0, ng = 0, nsh = 0, nterm = 0, npa = 0;
    int64_t nbox = 0, npts = 0;
    double h = 0.0, r0 = 0.0, t = 0.0;
    int32_t *cell = nullptr;
    double *lo = nullptr, *blo = nullptr, *bsz = nullptr, *tab = nullptr, *centers = nullptr;
    int64_t *bptr = nullptr, *pee_off = nullptr, *pair_ptr = nullptr;
    int32_t *item_slot = nullptr, *item_t0 = nullptr, *item_nt = nullptr, *pair_ij = nullptr,
            *pc = nullptr;
    double *Pee = nullptr, *Ptile = nullptr, *Pnn = nullptr;
    int32_t *item_q0 = nullptr, *item_qn = nullptr, *item_pi = nullptr;
    int32_t *f_slot = nullptr, *f_t0 = nullptr, *f_nt = nullptr, *f_p0 = nullptr, *f_np = nullptr;
    int32_t *nn_slot = nullptr, *nn_q0 = nullptr, *nn_qn = nullptr, *nn_pi = nullptr;
    int32_t *nnf_slot = nullptr, *nnf_p0 = nullptr, *nnf_np = nullptr;
    int n_nn = 0, n_nnf = 0;
    std::vector<int> batch_item, batch_pair, batch_fin;  // [nbatch + 1] each
  } ea;
  // self-consistent field quantities (chebfilter_scf_setup): the SCF cells
  // (plain cells, then the cells with an adaptive rule) with their point
  // ranges, the points' coordinates and weights, density-matrix work items
  // and batches, per-colour SCF cell lists, the Poisson system and the
  // mixing history
  struct {
    int nscf = 0, nplain = 0, nq = 0, cg_max = 0, depth = 0, nhist = 0, head = 0;
    int64_t P = 0, P_plain = 0;
    double cc[3] = {0.0, 0.0, 0.0}, cs = 1.0, cg_tol = 0.0, beta = 0.0;
    int32_t *cell = nullptr, *cna = nullptr, *seq = nullptr, *col_cells = nullptr;
    int32_t *dm_c = nullptr, *dm_t0 = nullptr, *dm_nt = nullptr;
    int32_t *rho_c = nullptr, *rho_t0 = nullptr, *rho_nt = nullptr, *rho_q0 = nullptr;
    std::vector<int> rho_off;                     // per batch and range index: first item
    int64_t *pofs = nullptr, *pcnt = nullptr, *doff = nullptr;
    double *lo = nullptr, *xyz = nullptr, *w = nullptr, *Dbuf = nullptr, *f2 = nullptr;
    int64_t f2_cap = 0;
    double *A = nullptr, *dinv = nullptr, *pb = nullptr, *px = nullptr, *pr = nullptr,
           *pz = nullptr, *pp = nullptr, *pq = nullptr, *vxc = nullptr, *part = nullptr,
           *dot = nullptr, *hin = nullptr, *hF = nullptr;
    std::vector<int> dm_item, dm_cell, col_ofs;   // batches' first item / first SCF cell; colours
    std::vector<int32_t> plain_cells;
    std::vector<double> gram;                     // depth x depth, weighted residual products
  } scf;
  rocblas_handle rb = nullptr;
  std::string err;
  bool profiling = false;
  std::map<std::string, ProfEntry> prof;
  std::vector<void *> allocs;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static cf_status set_err(cf_ctx *c, cf_status st, const std::string &msg) {
  if (c) c->err = msg; else g_init_error = msg;
  return st;
}

#define HIPCHK(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return set_err(ctx, CF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define STCHK(call)                     \
  do {                                  \
    cf_status s_ = (call);              \
    if (s_ != CF_OK) return s_;         \
  } while (0)

template <typename T>
static cf_status dalloc(cf_ctx *c, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, CF_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return CF_OK;
}

// Event-timed kernel family (only when profiling is on); `flops` is the
// algorithmic work credited to the bracketed launches.
struct Scope {
  cf_ctx *c;
  const char *name;
  double flops;
  hipEvent_t a = nullptr, b = nullptr;
  Scope(cf_ctx *c_, const char *n, double f = 0.0) : c(c_), name(n), flops(f) {
    if (c->profiling && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, c->stream);
  }
  ~Scope() {
    if (c->profiling && a && b) {
      (void)hipEventRecord(b, c->stream);
      ProfEntry &pe = c->prof[name];
      pe.pending.emplace_back(a, b);
      pe.flops += flops;
    }
  }
};

static cf_status check_block(cf_ctx *c, const void *X, int64_t ldx, int64_t N, const char *nm) {
  if (N < 0 || N > c->max_cols)
    return set_err(c, N < 0 ? CF_EINVAL : CF_ENOMEM,
                   std::string(nm) + ": N out of range [0, max_cols]");
  if (N > 0 && (X == nullptr || ldx < N))
    return set_err(c, CF_EINVAL, std::string(nm) + ": null block or ld < N");
  return CF_OK;
}

// ---------------------------------------------------------------------------
// operator cores (all enqueue on c->stream)
// ---------------------------------------------------------------------------
// Classical elemental products R' = H^cc X over all colours (Y rows 0..n_h).
// With a finishing step, DOFs outside the enriched region take the recurrence
// in the cell kernel and their rows of Y are not written.
static cf_status core_cells(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy, int N,
                            const CellFinish &f = CellFinish()) {
  for (size_t k = 0; k + 1 < c->col_off.size(); ++k) {
    // elemental dense product: 2 npc^2 N flops per cell (single columns run the
    // VALU kernel k_cell_gemv, timed under their own name)
    Scope sc(c, N == 1 ? "cell_gemv" : "cell_gemm",
             2.0 * c->npc * c->npc * (double)N * (c->col_off[k + 1] - c->col_off[k]));
    HIPCHK(c, launch_cell_gemm(c->stream, c->Hp, c->dofp, c->flagp, c->cells + c->col_off[k],
                               c->col_off[k + 1] - c->col_off[k], X, ldx, Y, ldy, N, f));
  }
  return CF_OK;
}

static EpiArgs epi_base(cf_ctx *c, int N) {
  EpiArgs g;
  g.n_h = c->n_h;
  g.n_e = c->n_e;
  g.N = N;
  if (c->n_e > 0) {
    g.qptr = c->qptr;
    g.qmax = c->qmax;
    g.qidx = c->qidx;
    g.Q = c->Q;
    g.ldq = c->ldw;
  }
  return g;
}

// Q = cell-local transposed coupling products (see k_enr_q).
static cf_status core_enr_q(cf_ctx *c, const double *U, int64_t ldu, double cU, const double *V,
                            int64_t ldv, double cV, int N) {
  Scope sc(c, "enr_q");
  HIPCHK(c, launch_enr_q(c->stream, c->Hec, c->Mec, c->eptr, c->eidx, c->ecells, c->epos_part,
                         c->necells, c->kmax,
                         U, ldu, cU, V, ldv, cV, c->Q, c->ldw, N));
  return CF_OK;
}

// Y = H^E X (Eq. H2x2): Y_c = H^cc X_c + H^ec^T X_e, Y_e = H^ec X_c + H^ee X_e.
static cf_status core_apply_H(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                              int N) {
  STCHK(core_cells(c, X, ldx, Y, ldy, N));
  if (c->n_e == 0) return CF_OK;
  const double *Xe = X + c->n_h * ldx;
  double *Ye = Y + c->n_h * ldy;
  {
    Scope sc(c, "enr_gemm");
    HIPCHK(c, launch_enr_part(c->stream, c->HT, c->MT, c->toff, c->tld, c->eptr, c->dofp, c->ecells_part,
                              c->necells, c->epitems, c->nepitems, X, ldx, 1.0, nullptr, 0, nullptr, 0.0, c->P, c->ldw,
                              N));
    HIPCHK(c, launch_enr_reduce(c->stream, (int)c->n_e, c->aptr, c->alist, c->P, c->ldw, 1.0,
                                nullptr, 0, 0.0, c->Hee, Xe, ldx, Ye, ldy, N));
  }
  STCHK(core_enr_q(c, Xe, ldx, 1.0, nullptr, 0, 0.0, N));
  EpiArgs g = epi_base(c, N);
  g.R = Y; g.ldr = ldy;
  g.Ee = Ye; g.lde = ldy;
  g.Out = Y; g.ldo = ldy;
  Scope sc(c, "epilogue");
  HIPCHK(c, launch_epilogue(c->stream, g));
  return CF_OK;
}

// Y = M^E X (Eq. M2x2): Y_c = D X_c + M^ec^T X_e, Y_e = M^ec X_c + M^ee X_e.
static cf_status core_apply_M(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                              int N) {
  const double *Xe = X + c->n_h * ldx;
  double *Ye = Y + c->n_h * ldy;
  if (c->n_e > 0) {
    Scope sc(c, "enr_gemm");
    HIPCHK(c, launch_enr_part(c->stream, c->HT, c->MT, c->toff, c->tld, c->eptr, c->dofp, c->ecells_part,
                              c->necells, c->epitems, c->nepitems, nullptr, 0, 0.0, X, ldx, nullptr, 1.0, c->P, c->ldw,
                              N));
    HIPCHK(c, launch_enr_reduce(c->stream, (int)c->n_e, c->aptr, c->alist, c->P, c->ldw, 1.0,
                                nullptr, 0, 0.0, c->Mee, Xe, ldx, Ye, ldy, N));
    STCHK(core_enr_q(c, nullptr, 0, 0.0, Xe, ldx, 1.0, N));
  }
  EpiArgs g = epi_base(c, N);
  g.R = X; g.ldr = ldx; g.dR = c->dvec;
  g.Ee = Ye; g.lde = ldy;
  g.Out = Y; g.ldo = ldy;
  Scope sc(c, "epilogue");
  HIPCHK(c, launch_epilogue(c->stream, g));
  return CF_OK;
}

// z = S^-1 w into Zb, where w (in Wb) has been formed by the caller.
static cf_status core_schur_solve(cf_ctx *c, int N) {
  Scope sc(c, "enr_reduce");
  HIPCHK(c, launch_enr_reduce(c->stream, (int)c->n_e, c->aptr, c->alist, nullptr, 0, 0.0, nullptr, 0,
                              0.0, c->Sinv, c->Wb, c->ldw, c->Zb, c->ldw, N));
  return CF_OK;
}

// Y = (M^E)^-1 X (block-wise inverse, Sec. IV.D) for n <= ldw columns:
// w = x_e - M^ec D^-1 x_c, z = S^-1 w, y_c = D^-1 (x_c - M^ec^T z), y_e = z.
static cf_status core_apply_Sinv(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                                 int n) {
  if (c->n_e > 0) {
    Scope sc(c, "enr_gemm");
    HIPCHK(c, launch_enr_part(c->stream, c->HT, c->MT, c->toff, c->tld, c->eptr, c->dofp, c->ecells_part,
                              c->necells, c->epitems, c->nepitems, nullptr, 0, 0.0, X, ldx, c->dinv, -1.0, c->P, c->ldw,
                              n));
    HIPCHK(c, launch_enr_reduce(c->stream, (int)c->n_e, c->aptr, c->alist, c->P, c->ldw, 1.0,
                                X + c->n_h * ldx, ldx, 1.0, nullptr, nullptr, 0, c->Wb, c->ldw,
                                n));
    STCHK(core_schur_solve(c, n));
    STCHK(core_enr_q(c, nullptr, 0, 0.0, c->Zb, c->ldw, -1.0, n));
  }
  EpiArgs g = epi_base(c, n);
  g.R = X; g.ldr = ldx; g.dR = c->dinv; g.dC = c->dinv;
  g.Ee = c->Zb; g.lde = c->ldw;
  g.Out = Y; g.ldo = ldy;
  HIPCHK(c, launch_epilogue(c->stream, g));
  return CF_OK;
}

// Out = c1 * H~ Xin + c2 * Yk + c3 * Yp, H~ = (M^E)^-1 H^E, with the block-wise
// inverse of Sec. IV.D.  With R' = H^cc X_c and K = M^ec D^-1 H^ec^T (formed
// at init):  w = H^ec X_c - M^ec D^-1 R' + (H^ee - K) X_e,  z = S^-1 w,
// y_c = D^-1 (R' + H^ec^T X_e - M^ec^T z),  y_e = z; the two transposed
// coupling products go through the enriched-cell buffer Q.
static cf_status core_htilde_step(cf_ctx *c, const double *Xin, int64_t ldxin, int N, double c1,
                                  const double *Yk, int64_t ldyk, double c2, const double *Yp,
                                  int64_t ldyp, double c3, double *Out, int64_t ldo) {
  const int64_t ldr = c->ldw;
  // rows outside the enriched region are finished by the cell kernel (it holds
  // X = Y_k in LDS, so this needs Yk to be Xin or absent)
  const bool finish = Yk == nullptr || (Yk == Xin && ldyk == ldxin);
  CellFinish f;
  if (finish) {
    f.dinv = c->dinv;
    f.c1 = c1; f.c2 = Yk ? c2 : 0.0; f.c3 = Yp ? c3 : 0.0;
    f.Yp = Yp; f.ldyp = ldyp;
    f.Out = Out; f.ldo = ldo;
  }
  STCHK(core_cells(c, Xin, ldxin, c->R, ldr, N, f));
  const double *Xe = Xin + c->n_h * ldxin;
  if (c->n_e > 0) {
    {
      Scope sc(c, "enr_part");
      HIPCHK(c, launch_enr_part(c->stream, c->HT, c->MT, c->toff, c->tld, c->eptr, c->dofp,
                                c->ecells_part, c->necells, c->epitems, c->nepitems, Xin, ldxin,
                                1.0, c->R, ldr, c->dinv, -1.0, c->P, c->ldw, N));
    }
    {
      Scope sc(c, "enr_reduce");
      HIPCHK(c, launch_enr_reduce(c->stream, (int)c->n_e, c->aptr, c->alist, c->P, c->ldw, 1.0,
                                  nullptr, 0, 0.0, c->Hmod, Xe, ldxin, c->Wb, c->ldw, N));
    }
    STCHK(core_schur_solve(c, N));
    STCHK(core_enr_q(c, Xe, ldxin, 1.0, c->Zb, c->ldw, -1.0, N));
  }
  EpiArgs g = epi_base(c, N);
  g.R = c->R; g.ldr = ldr; g.dR = c->dinv; g.dC = c->dinv;
  g.Ee = c->Zb; g.lde = c->ldw;
  g.c1 = c1; g.Yk = Yk; g.ldyk = ldyk; g.c2 = c2; g.Yp = Yp; g.ldyp = ldyp; g.c3 = c3;
  g.Out = Out; g.ldo = ldo;
  if (finish) { g.rows = c->regrows; g.nrows = c->nregrows; }
  Scope sc(c, "epilogue");
  HIPCHK(c, launch_epilogue(c->stream, g));
  return CF_OK;
}

// Reduced-precision copies of the operator and FP32 workspace (once per
// context and precision).
static cf_status ensure_lowp(cf_ctx *c, bool bf16) {
  const int64_t mc = c->ldw;
  if (!c->F0) {
    STCHK(dalloc(c, &c->F0, (size_t)c->n * mc));
    STCHK(dalloc(c, &c->F1, (size_t)c->n * mc));
    STCHK(dalloc(c, &c->R32, (size_t)c->n_h * mc));
    if (c->n_e > 0) {
      STCHK(dalloc(c, &c->HT32, (size_t)std::max<int64_t>(c->ttot, 1)));
      STCHK(dalloc(c, &c->MT32, (size_t)std::max<int64_t>(c->ttot, 1)));
      STCHK(dalloc(c, &c->Hec32, (size_t)std::max<int64_t>(c->nnz, 1) * NPAD));
      STCHK(dalloc(c, &c->Mec32, (size_t)std::max<int64_t>(c->nnz, 1) * NPAD));
      STCHK(dalloc(c, &c->P32, (size_t)std::max<int64_t>(c->nnz, 1) * mc));
      STCHK(dalloc(c, &c->Q32, (size_t)std::max<int>(c->necells, 1) * NPAD * mc));
      HIPCHK(c, launch_to_f32(c->stream, c->ttot, c->HT, c->HT32));
      HIPCHK(c, launch_to_f32(c->stream, c->ttot, c->MT, c->MT32));
      HIPCHK(c, launch_to_f32(c->stream, c->nnz * NPAD, c->Hec, c->Hec32));
      HIPCHK(c, launch_to_f32(c->stream, c->nnz * NPAD, c->Mec, c->Mec32));
    }
  }
  const int64_t hsz = c->E * NPAD * NPAD;
  if (bf16 && !c->Hp16) {
    uint16_t *h = nullptr;
    STCHK(dalloc(c, &h, (size_t)hsz));
    c->Hp16 = h;
    HIPCHK(c, launch_to_bf16(c->stream, hsz, c->Hp, c->Hp16));
  }
  if (!c->Hp32) {   // both forms (the BF16 form for the cells near the enriched region)
    STCHK(dalloc(c, &c->Hp32, (size_t)hsz));
    HIPCHK(c, launch_to_f32(c->stream, hsz, c->Hp, c->Hp32));
  }
  return CF_OK;
}

// Scale bookkeeping for a reduced filter of degree m.
static cf_status ensure_lp_scale(cf_ctx *c, int m) {
  if (m + 2 <= c->lp_cap) return CF_OK;
  const int cap = std::max(256, m + 2);
  STCHK(dalloc(c, &c->lp_mx, (size_t)cap * MX_SLOTS));
  STCHK(dalloc(c, &c->lp_s, (size_t)cap));
  STCHK(dalloc(c, &c->lp_mult, (size_t)2 * cap));
  c->lp_cap = cap;
  return CF_OK;
}

// FP32 form of core_htilde_step with the finishing step always on:
//   Out = c1 * H~ Xin + c2 * Xin + c3 * Yp
// Elemental and coupling products in FP32 (cell matrices FP32 or BF16 with
// FP32 accumulation); the enrichment-row sums, the Schur solve z = S^-1 w and
// z itself stay FP64.  Out may be Yp (each element is read before it is
// written, by the same thread).
static cf_status core_htilde_step_lp(cf_ctx *c, bool bf16, const float *Xin, int64_t ldxin, int N,
                                     float c1, float c2, const float *Yp, int64_t ldyp, float c3,
                                     float *Out, int64_t ldo, const float *mult, unsigned *mx) {
  const int64_t mc = c->ldw;
  CellFinishF f;
  f.dinv = c->dinv;
  f.c1 = c1; f.c2 = c2; f.c3 = Yp ? c3 : 0.f;
  f.Yp = Yp; f.ldyp = ldyp;
  f.Out = Out; f.ldo = ldo;
  f.mult = mult; f.mx = mx;
  const double fl = 2.0 * c->npc * c->npc * (double)N;
  for (size_t k = 0; k + 1 < c->col_off.size(); ++k) {
    const int c0 = c->col_off[k], cnt = c->col_off[k + 1] - c0;
    // cells of one colour share no DOF, so the colour may go in two launches
    const int nfp = bf16 ? c->near_cnt[k] : cnt;
    if (nfp > 0) {
      Scope sc(c, "cell_gemm_fp32", fl * nfp);
      HIPCHK(c, launch_cell_gemm_lp(c->stream, false, c->lp_nsb[0], c->Hp32, c->dofp, c->flagp,
                                    c->cells_split + c0, nfp, Xin, ldxin, c->R32, mc, N, f));
    }
    if (cnt - nfp > 0) {
      Scope sc(c, "cell_gemm_bf16", fl * (cnt - nfp));
      HIPCHK(c, launch_cell_gemm_lp(c->stream, true, c->lp_nsb[1], c->Hp16, c->dofp, c->flagp,
                                    c->cells_split + c0 + nfp, cnt - nfp, Xin, ldxin, c->R32, mc, N,
                                    f));
    }
  }
  const float *Xe = Xin + c->n_h * ldxin;
  if (c->n_e > 0) {
    {
      Scope sc(c, "enr_part");
      HIPCHK(c, launch_enr_part_f32(c->stream, c->HT32, c->MT32, c->toff, c->tld, c->eptr, c->dofp,
                                    c->ecells_part, c->necells, Xin, ldxin, 1.f, c->R32, mc, c->dinv,
                                    -1.f, c->P32, mc, N, c->lp_bmap));
    }
    {
      Scope sc(c, "enr_reduce");
      HIPCHK(c, launch_enr_reduce_f32(c->stream, (int)c->n_e, c->aptr, c->alist, c->P32, mc,
                                      c->Hmod, Xe, ldxin, c->Wb, mc, N));
    }
    STCHK(core_schur_solve(c, N));
    {
      Scope sc(c, "enr_q");
      HIPCHK(c, launch_enr_q_f32(c->stream, c->Hec32, c->Mec32, c->eptr, c->eidx, c->ecells,
                                 c->epos_part,
                                 c->necells, c->kmax, Xe, ldxin, 1.f, c->Zb, mc, -1.f, c->Q32, mc,
                                 N));
    }
  }
  EpiArgsF g;
  g.n_h = c->n_h; g.n_e = c->n_e; g.N = N;
  g.rows = c->regrows; g.nrows = c->nregrows;
  g.dinv = c->dinv;
  g.R = c->R32; g.ldr = mc;
  if (c->n_e > 0) { g.qptr = c->qptr; g.qidx = c->qidx; g.Q = c->Q32; g.ldq = mc; }
  g.Ee = c->Zb; g.lde = mc;
  g.c1 = c1; g.Yk = Xin; g.ldyk = ldxin; g.c2 = c2;
  g.Yp = Yp; g.ldyp = ldyp; g.c3 = Yp ? c3 : 0.f;
  g.Out = Out; g.ldo = ldo;
  g.mult = mult; g.mx = mx;
  Scope sc(c, "epilogue");
  HIPCHK(c, launch_epilogue_f32(c->stream, g));
  return CF_OK;
}

// Out = In * W for row-major n x N blocks and a row-major N x N W (ld N):
// a plain library GEMM (column-major view: Out^T = W^T In^T).  In == Out
// (same ld) rotates in place by row blocks through the work block T, viewed
// as rb x N with rb = n ldw / N rows (one block when N <= ldw).
static cf_status core_rotate(cf_ctx *c, const double *In, int64_t ldi, const double *W, int N,
                             double *Out, int64_t ldo) {
  Scope sc(c, "rotate", 2.0 * (double)c->n * N * N);
  const double one = 1.0, zero = 0.0;
  rocblas_set_pointer_mode(c->rb, rocblas_pointer_mode_host);
  if (In != Out) {
    if (rocblas_dgemm(c->rb, rocblas_operation_none, rocblas_operation_none, N, (rocblas_int)c->n,
                      N, &one, W, N, In, (rocblas_int)ldi, &zero, Out, (rocblas_int)ldo) !=
        rocblas_status_success)
      return set_err(c, CF_EDEVICE, "rotate: rocblas_dgemm failed");
    return CF_OK;
  }
  if (ldi != ldo) return set_err(c, CF_EINVAL, "rotate: in-place rotation needs one leading dimension");
  const int64_t rb = std::max<int64_t>(1, std::min<int64_t>(c->n, (c->n * c->ldw) / N));
  for (int64_t r0 = 0; r0 < c->n; r0 += rb) {
    const int64_t rows = std::min(rb, c->n - r0);
    if (rocblas_dgemm(c->rb, rocblas_operation_none, rocblas_operation_none, N, (rocblas_int)rows,
                      N, &one, W, N, In + r0 * ldi, (rocblas_int)ldi, &zero, c->T, N) !=
        rocblas_status_success)
      return set_err(c, CF_EDEVICE, "rotate: rocblas_dgemm failed");
    HIPCHK(c, launch_copy(c->stream, rows, N, c->T, N, Out + r0 * ldo, ldo));
  }
  return CF_OK;
}

// Gram G = A^T B (N x N, ld N) through the chunked partial kernel.
static cf_status core_gram(cf_ctx *c, const double *A, int64_t lda, const double *B, int64_t ldb,
                           int64_t nrows, int N, double *Gout, int mode) {
  Scope sc(c, "gram");
  const int nch = c->gp_chunks;
  const int64_t chunk_rows = (nrows + nch - 1) / nch;
  HIPCHK(c, launch_gram_partial(c->stream, A, lda, B, ldb, nrows, N, N, nch, chunk_rows, c->Gp,
                                mode));
  HIPCHK(c, launch_gram_reduce(c->stream, c->Gp, nch, N, N, Gout, N, mode));
  return CF_OK;
}

// Slab of a Gram matrix: G[i][j] (ld ldg) = (A^T B)[i][j], i < Na, j < Nb.
static cf_status core_gram_slab(cf_ctx *c, const double *A, int64_t lda, int Na, const double *B,
                                int64_t ldb, int Nb, double *Gout, int64_t ldg) {
  Scope sc(c, "gram");
  const int nch = c->gp_chunks;
  const int64_t chunk_rows = (c->n + nch - 1) / nch;
  HIPCHK(c, launch_gram_partial(c->stream, A, lda, B, ldb, c->n, Na, Nb, nch, chunk_rows, c->Gp,
                                GRAM_FULL));
  HIPCHK(c, launch_gram_reduce(c->stream, c->Gp, nch, Na, Nb, Gout, ldg, GRAM_FULL));
  return CF_OK;
}

// One Cholesky-QR pass In -> Out (Out = In * S * L^-T, G' = S In^T In S = L L^T).
static cf_status core_cholqr_pass(cf_ctx *c, const double *In, int64_t ldi, double *Out,
                                  int64_t ldo, int N, double shift, int *failed) {
  STCHK(core_gram(c, In, ldi, In, ldi, c->n, N, c->G, GRAM_UPPER));
  // scaled, shifted Gram (our kernel), then the library Cholesky: on the
  // row-major G, the column-major upper factor is the row-major lower L
  HIPCHK(c, hipMemsetAsync(c->flag, 0, 2 * sizeof(int), c->stream));
  HIPCHK(c, launch_chol_scale(c->stream, c->G, N, shift, c->sv, c->flag));
  {
    Scope sc(c, "cholesky");
    if (rocsolver_dpotrf(c->rb, rocblas_fill_upper, N, c->G, N, (rocblas_int *)(c->flag + 1)) !=
        rocblas_status_success)
      return set_err(c, CF_EDEVICE, "cholqr: rocsolver_dpotrf failed");
  }
  int h_flag[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(h_flag, c->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *failed = h_flag[0] | h_flag[1];
  if (*failed) return CF_OK;
  HIPCHK(c, launch_tri_inv_T(c->stream, c->G, c->sv, N, c->Wm));
  return core_rotate(c, In, ldi, c->Wm, N, Out, ldo);
}

// Orthonormalise In into Out through the scratch blocks T and R (In may equal
// Out; Out must not be T or R).  Blocks wider than the work blocks are
// orthonormalised in place in Out (every pass rotates by row blocks).
static cf_status core_cholqr(cf_ctx *c, const double *In, int64_t ldi, double *Out, int64_t ldo,
                             int N) {
  const int64_t ldt = c->ldw;
  int failed = 0;
  if (N > ldt) {
    if (In != Out) HIPCHK(c, launch_copy(c->stream, c->n, N, In, ldi, Out, ldo));
    STCHK(core_cholqr_pass(c, Out, ldo, Out, ldo, N, 0.0, &failed));
    if (failed) {
      const double u = 1.1102230246251565e-16;
      const double shift = 11.0 * ((double)c->n * N + (double)N * (N + 1)) * u * N;
      STCHK(core_cholqr_pass(c, Out, ldo, Out, ldo, N, shift, &failed));
      if (failed)
        return set_err(c, CF_ENOTSPD, "cholqr: Gram matrix not positive definite even with shift");
      STCHK(core_cholqr_pass(c, Out, ldo, Out, ldo, N, 0.0, &failed));
      if (failed) return set_err(c, CF_ENOTSPD, "cholqr: second pass failed after shift");
    }
    STCHK(core_cholqr_pass(c, Out, ldo, Out, ldo, N, 0.0, &failed));
    if (failed) return set_err(c, CF_ENOTSPD, "cholqr: second pass not positive definite");
    return CF_OK;
  }
  STCHK(core_cholqr_pass(c, In, ldi, c->T, ldt, N, 0.0, &failed));
  if (failed) {
    // shifted Cholesky-QR: shift of the unit-diagonal Gram by 11 (nN + N(N+1)) u N
    const double u = 1.1102230246251565e-16;
    const double shift = 11.0 * ((double)c->n * N + (double)N * (N + 1)) * u * N;
    STCHK(core_cholqr_pass(c, In, ldi, c->T, ldt, N, shift, &failed));
    if (failed)
      return set_err(c, CF_ENOTSPD, "cholqr: Gram matrix not positive definite even with shift");
    STCHK(core_cholqr_pass(c, c->T, ldt, c->R, ldt, N, 0.0, &failed));
    if (failed) return set_err(c, CF_ENOTSPD, "cholqr: second pass failed after shift");
    STCHK(core_cholqr_pass(c, c->R, ldt, Out, ldo, N, 0.0, &failed));
  } else {
    STCHK(core_cholqr_pass(c, c->T, ldt, Out, ldo, N, 0.0, &failed));
  }
  if (failed) return set_err(c, CF_ENOTSPD, "cholqr: second pass not positive definite");
  return CF_OK;
}

static cf_status check_out_finite(cf_ctx *c, const double *Y, int64_t ldy, int N, const char *nm) {
  if (!c->check_finite || N == 0) return CF_OK;
  HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  HIPCHK(c, launch_check_finite(c->stream, Y, ldy, c->n, N, c->flag));
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (h) return set_err(c, CF_ENUMERIC, std::string(nm) + ": non-finite values in the output");
  return CF_OK;
}

// k Lanczos steps of M^-1 H from v0, enqueued on the context's stream with no
// host wait; the two bounds (lowest Ritz value, upper bound) land in out[0..1]
// (device memory).
static cf_status core_lanczos(cf_ctx *c, const double *v0, int k, double *out) {
  const int64_t n = c->n;
  double *vprev = c->lzv, *v = c->lzv + n, *w = c->lzv + 2 * n, *mv = c->lzv + 3 * n;
  double *coef = c->lzcoef;
  const int nblk = 512;
  HIPCHK(c, launch_fill(c->stream, coef, 2 * 64 + 8, 0.0));
  STCHK(core_apply_M(c, v0, 1, mv, 1, 1));
  HIPCHK(c, launch_dot(c->stream, n, v0, mv, coef, c->lzpart, nblk));
  HIPCHK(c, launch_lanczos_update(c->stream, n, 0, const_cast<double *>(v0), nullptr, nullptr, coef,
                                  v, nullptr, nblk, 0));
  for (int j = 0; j < k; ++j) {
    STCHK(core_htilde_step(c, v, 1, 1, 1.0, nullptr, 0, 0.0, nullptr, 0, 0.0, w, 1));
    if (j > 0)
      HIPCHK(c, launch_lanczos_update(c->stream, n, j, w, v, vprev, coef, nullptr, nullptr, nblk, 1));
    STCHK(core_apply_M(c, v, 1, mv, 1, 1));
    HIPCHK(c, launch_dot(c->stream, n, w, mv, coef + 1 + 2 * j, c->lzpart, nblk));
    HIPCHK(c, launch_lanczos_update(c->stream, n, j, w, v, vprev, coef, nullptr, nullptr, nblk, 2));
    STCHK(core_apply_M(c, w, 1, mv, 1, 1));
    HIPCHK(c, launch_dot(c->stream, n, w, mv, coef + 2 + 2 * j, c->lzpart, nblk));
    if (j + 1 < k) {
      HIPCHK(c, launch_lanczos_update(c->stream, n, j, w, v, vprev, coef, vprev, nullptr, nblk, 3));
      std::swap(vprev, v);   // vprev <- old v, v <- new vector
    }
  }
  HIPCHK(c, launch_tridiag_bounds(c->stream, coef, nullptr, k, out));
  return CF_OK;
}

static void free_ctx(cf_ctx *c) {
  if (!c) return;
  if (c->rb) rocblas_destroy_handle(c->rb);
  for (auto &kv : c->prof)
    for (auto &ev : kv.second.pending) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  for (void *q : c->allocs) (void)hipFree(q);
  delete c;
}

// Cell matrices H_cc (host, [E][npc][npc]) -> c->Hp, padded to NPAD x NPAD and
// symmetrised after checking symmetry to 1e-10 of the block's largest entry;
// refreshes the reduced-precision copies when they exist.
static cf_status upload_cells(cf_ctx *c, const double *H_cc, const char *who) {
  const int64_t E = c->E;
  const int npc = c->npc;
  const int64_t batch = 256;
  std::vector<double> buf((size_t)batch * NPAD * NPAD);
  for (int64_t e0 = 0; e0 < E; e0 += batch) {
    const int64_t nb = std::min(batch, E - e0);
    std::fill(buf.begin(), buf.begin() + nb * NPAD * NPAD, 0.0);
    for (int64_t b = 0; b < nb; ++b) {
      const double *H = H_cc + (e0 + b) * npc * npc;
      double *o = buf.data() + b * NPAD * NPAD;
      double hmax = 0.0;
      for (int64_t q = 0; q < (int64_t)npc * npc; ++q) {
        if (!std::isfinite(H[q])) return set_err(c, CF_EINVAL, std::string(who) + ": non-finite H_cc");
        hmax = std::max(hmax, std::fabs(H[q]));
      }
      for (int a = 0; a < npc; ++a)
        for (int bb = 0; bb < npc; ++bb) {
          const double x = H[a * npc + bb], y = H[bb * npc + a];
          if (std::fabs(x - y) > 1e-10 * hmax)
            return set_err(c, CF_EINVAL, std::string(who) + ": H_cc block not symmetric");
          o[a * NPAD + bb] = 0.5 * (x + y);
        }
    }
    // ordered after earlier work on the context's stream that reads Hp
    HIPCHK(c, hipMemcpyAsync(c->Hp + e0 * NPAD * NPAD, buf.data(), nb * NPAD * NPAD * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  const int64_t hsz = E * NPAD * NPAD;
  if (c->Hp32) HIPCHK(c, launch_to_f32(c->stream, hsz, c->Hp, c->Hp32));
  if (c->Hp16) HIPCHK(c, launch_to_bf16(c->stream, hsz, c->Hp, c->Hp16));
  return CF_OK;
}

// ---------------------------------------------------------------------------
// Fixed device scratch of chebfilter_lanczos_bounds_noalloc: a file-scope
// device array (each GPU holds its own copy from module load until the
// process ends).  Host code never uses the array's name as an address: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current.
// ---------------------------------------------------------------------------
static constexpr int64_t NOALLOC_DOUBLES = (64ll << 20) / 8;     // 64 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_addr;     // device ordinal -> its copy of scratch
}  // namespace

static cf_status scratch_address(cf_ctx *c, double **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(c->device);
  if (it != g_scratch_addr.end()) { *out = it->second; return CF_OK; }
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return set_err(c, CF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_addr[c->device] = static_cast<double *>(ptr);
  *out = static_cast<double *>(ptr);
  return CF_OK;
}

static int64_t align32(int64_t x) { return (x + 31) / 32 * 32; }   // 256-byte pieces

// Doubles of scratch one single-vector Lanczos run needs: the work rows R (n),
// the four Lanczos vectors (4n), coupling partials (one per coupling row),
// the enriched-cell buffer (NPAD per enriched cell), w and z (n_e each), the
// tridiagonal coefficients and the dot-product partials.
static int64_t noalloc_need(const cf_ctx *c) {
  return align32(c->n) + align32(4 * c->n) + align32(std::max<int64_t>(c->nnz, 1)) +
         align32((int64_t)std::max(c->necells, 1) * NPAD) + 2 * align32(std::max<int64_t>(c->n_e, 1)) +
         align32(2 * 64 + 8) + align32(1024);
}

// Points the context's single-column work buffers into the scratch (leading
// dimension 1) for the lifetime of the object, then restores them.
struct ScratchWork {
  cf_ctx *c;
  double *R, *P, *Q, *Wb, *Zb, *lzv, *lzcoef, *lzpart;
  int64_t ldw;
  ScratchWork(cf_ctx *c_, double *base) : c(c_) {
    R = c->R; P = c->P; Q = c->Q; Wb = c->Wb; Zb = c->Zb;
    lzv = c->lzv; lzcoef = c->lzcoef; lzpart = c->lzpart; ldw = c->ldw;
    double *q = base;
    auto take = [&](int64_t count) { double *r = q; q += align32(count); return r; };
    c->R = take(c->n);
    c->lzv = take(4 * c->n);
    c->P = take(std::max<int64_t>(c->nnz, 1));
    c->Q = take((int64_t)std::max(c->necells, 1) * NPAD);
    c->Wb = take(std::max<int64_t>(c->n_e, 1));
    c->Zb = take(std::max<int64_t>(c->n_e, 1));
    c->lzcoef = take(2 * 64 + 8);
    c->lzpart = take(1024);
    c->ldw = 1;
  }
  ~ScratchWork() {
    c->R = R; c->P = P; c->Q = Q; c->Wb = Wb; c->Zb = Zb;
    c->lzv = lzv; c->lzcoef = lzcoef; c->lzpart = lzpart; c->ldw = ldw;
  }
};

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
static cf_status do_init(const cf_problem *pr, const cf_options *opt, cf_ctx *c) {
  if (!pr || !opt) return set_err(c, CF_EINVAL, "init: null problem or options");
  if (pr->p < 1 || pr->p > 4) return set_err(c, CF_EINVAL, "init: element degree must be 1..4");
  const int npc = (pr->p + 1) * (pr->p + 1) * (pr->p + 1);
  if (pr->n_cells < 1 || pr->n_h < 1 || pr->n_e < 0 || pr->n_h > (int64_t)INT32_MAX - 1 ||
      pr->n_cells > (int64_t)INT32_MAX)
    return set_err(c, CF_EINVAL, "init: bad sizes");
  if (!pr->cell_dof || !pr->H_cc || !pr->M_cc_diag)
    return set_err(c, CF_EINVAL, "init: null classical arrays");
  if (pr->n_e > 0 && (!pr->enr_ptr || !pr->enr_idx || !pr->H_ec || !pr->M_ec || !pr->H_ee || !pr->M_ee))
    return set_err(c, CF_EINVAL, "init: null enrichment arrays");
  if (opt->max_cols < 1) return set_err(c, CF_EINVAL, "init: max_cols must be >= 1");
  if (opt->col_chunk < 0) return set_err(c, CF_EINVAL, "init: col_chunk must be >= 0");
  c->device = opt->device;
  c->stream = (hipStream_t)opt->stream;
  c->check_finite = opt->check_finite;
  c->p = pr->p;
  c->npc = npc;
  c->E = pr->n_cells;
  c->n_h = pr->n_h;
  c->n_e = pr->n_e;
  c->n = pr->n_h + pr->n_e;
  c->max_cols = opt->max_cols;
  c->chunk = (opt->col_chunk > 0 && opt->col_chunk < opt->max_cols) ? opt->col_chunk : opt->max_cols;
  c->ldw = (c->chunk + 15) / 16 * 16;
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t E = c->E, n_h = c->n_h, n_e = c->n_e;

  // ---- classical validation, colouring and first-touch flags
  std::vector<int32_t> dof((size_t)E * NPAD, -1);
  std::vector<int> cover(n_h, 0);
  for (int64_t e = 0; e < E; ++e) {
    for (int a = 0; a < npc; ++a) {
      const int64_t d = pr->cell_dof[e * npc + a];
      if (d < -1 || d >= n_h) return set_err(c, CF_EINVAL, "init: cell_dof out of range");
      dof[e * NPAD + a] = (int32_t)d;
      if (d >= 0) {
        if (cover[d] == (int)e + 1) return set_err(c, CF_EINVAL, "init: repeated DOF within a cell");
        cover[d] = (int)e + 1;
      }
    }
  }
  for (int64_t d = 0; d < n_h; ++d)
    if (cover[d] == 0) return set_err(c, CF_EINVAL, "init: a free DOF belongs to no cell");
  for (int64_t d = 0; d < n_h; ++d) {
    const double v = pr->M_cc_diag[d];
    if (!(v > 0.0) || !std::isfinite(v)) return set_err(c, CF_EINVAL, "init: M_cc_diag must be > 0");
  }
  std::vector<uint64_t> used(n_h, 0);
  std::vector<int> colour(E);
  int ncol = 0;
  for (int64_t e = 0; e < E; ++e) {
    uint64_t mask = 0;
    for (int a = 0; a < npc; ++a) {
      const int32_t d = dof[e * NPAD + a];
      if (d >= 0) mask |= used[d];
    }
    if (~mask == 0) return set_err(c, CF_EINVAL, "init: cell graph needs more than 64 colours");
    const int col = __builtin_ctzll(~mask);
    colour[e] = col;
    ncol = std::max(ncol, col + 1);
    for (int a = 0; a < npc; ++a) {
      const int32_t d = dof[e * NPAD + a];
      if (d >= 0) used[d] |= (1ull << col);
    }
  }
  std::vector<int32_t> order;
  order.reserve(E);
  c->col_off.assign(1, 0);
  for (int col = 0; col < ncol; ++col) {
    for (int64_t e = 0; e < E; ++e)
      if (colour[e] == col) order.push_back((int32_t)e);
    c->col_off.push_back((int)order.size());
  }
  std::vector<uint8_t> first((size_t)E * NPAD, 0);
  {
    std::vector<uint8_t> touched(n_h, 0);
    for (int32_t e : order)
      for (int a = 0; a < npc; ++a) {
        const int32_t d = dof[(int64_t)e * NPAD + a];
        if (d >= 0 && !touched[d]) { touched[d] = 1; first[(int64_t)e * NPAD + a] = 1; }
      }
  }
  // last touch of each DOF in launch order (for the finishing step)
  std::vector<int64_t> last_slot(n_h, -1);
  for (int32_t e : order)
    for (int a = 0; a < npc; ++a) {
      const int32_t d = dof[(int64_t)e * NPAD + a];
      if (d >= 0) last_slot[d] = (int64_t)e * NPAD + a;
    }
  STCHK(dalloc(c, &c->dofp, dof.size()));
  STCHK(dalloc(c, &c->flagp, first.size()));
  STCHK(dalloc(c, &c->cells, order.size()));
  HIPCHK(c, hipMemcpy(c->dofp, dof.data(), dof.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->cells, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));

  // ---- cell matrices: padded to NPAD x NPAD, symmetrised, checked
  STCHK(dalloc(c, &c->Hp, (size_t)E * NPAD * NPAD));
  STCHK(upload_cells(c, pr->H_cc, "init"));
  {
    std::vector<double> dv(pr->M_cc_diag, pr->M_cc_diag + n_h), di(n_h);
    for (int64_t d = 0; d < n_h; ++d) di[d] = 1.0 / dv[d];
    STCHK(dalloc(c, &c->dvec, n_h));
    STCHK(dalloc(c, &c->dinv, n_h));
    HIPCHK(c, hipMemcpy(c->dvec, dv.data(), n_h * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->dinv, di.data(), n_h * sizeof(double), hipMemcpyHostToDevice));
  }

  // ---- workspace: n x ldw work blocks; N x N dense matrices (N <= max_cols)
  const int64_t mc = c->max_cols, lw = c->ldw;
  STCHK(dalloc(c, &c->R, (size_t)c->n * lw));
  STCHK(dalloc(c, &c->B2, (size_t)c->n * lw));
  STCHK(dalloc(c, &c->T, (size_t)c->n * lw));
  STCHK(dalloc(c, &c->U, (size_t)c->n * lw));
  {
    // Gram partial buffer: chunks of at least 512 rows, a multiple of 8 chunks,
    // at most 256, at most ~512 MB (small problems still fill the chip)
    int64_t nch = std::max<int64_t>(8, std::min<int64_t>(256, (c->n + 511) / 512));
    const int64_t cap = (int64_t)(512ll << 20) / (8 * mc * mc);
    nch = std::min<int64_t>(nch, std::max<int64_t>(8, cap));
    nch = (nch + 7) / 8 * 8;
    c->gp_chunks = (int)nch;
    STCHK(dalloc(c, &c->Gp, (size_t)nch * mc * mc));
  }
  STCHK(dalloc(c, &c->G, (size_t)mc * mc));
  STCHK(dalloc(c, &c->Wm, (size_t)mc * mc));
  STCHK(dalloc(c, &c->Wt, (size_t)mc * mc));
  STCHK(dalloc(c, &c->Hh, (size_t)mc * mc));
  STCHK(dalloc(c, &c->Mh, (size_t)mc * mc));
  STCHK(dalloc(c, &c->sv, (size_t)std::max<int64_t>(mc, n_e)));
  STCHK(dalloc(c, &c->theta, (size_t)mc));
  STCHK(dalloc(c, &c->evE, (size_t)mc));
  STCHK(dalloc(c, &c->flag, 4));
  STCHK(dalloc(c, &c->info, 4));
  STCHK(dalloc(c, &c->lzv, (size_t)c->n * 4));
  STCHK(dalloc(c, &c->lzcoef, 2 * 64 + 8));
  STCHK(dalloc(c, &c->lzpart, 1024));
  if (rocblas_create_handle(&c->rb) != rocblas_status_success)
    return set_err(c, CF_EDEVICE, "init: rocblas_create_handle failed");
  rocblas_set_stream(c->rb, c->stream);

  // ---- enrichment data
  c->col_off.shrink_to_fit();
  if (n_e > 0) {
    const int64_t *ep = pr->enr_ptr;
    if (ep[0] != 0) return set_err(c, CF_EINVAL, "init: enr_ptr[0] must be 0");
    int kmax = 0;
    for (int64_t e = 0; e < E; ++e) {
      if (ep[e + 1] < ep[e]) return set_err(c, CF_EINVAL, "init: enr_ptr not monotone");
      kmax = std::max<int>(kmax, (int)(ep[e + 1] - ep[e]));
    }
    c->kmax = kmax;
    const int64_t nnz = ep[E];
    c->nnz = nnz;
    std::vector<int32_t> eidx(std::max<int64_t>(nnz, 1));
    {
      std::vector<int64_t> seen(n_e, -1);
      for (int64_t e = 0; e < E; ++e)
        for (int64_t k = ep[e]; k < ep[e + 1]; ++k) {
          const int64_t al = pr->enr_idx[k];
          if (al < 0 || al >= n_e) return set_err(c, CF_EINVAL, "init: enr_idx out of range");
          if (seen[al] == e) return set_err(c, CF_EINVAL, "init: repeated enrichment index in a cell");
          seen[al] = e;
          eidx[k] = (int32_t)al;
        }
    }
    for (int64_t q = 0; q < nnz * npc; ++q)
      if (!std::isfinite(pr->H_ec[q]) || !std::isfinite(pr->M_ec[q]))
        return set_err(c, CF_EINVAL, "init: non-finite H_ec / M_ec");
    for (int64_t q = 0; q < n_e * n_e; ++q)
      if (!std::isfinite(pr->H_ee[q]) || !std::isfinite(pr->M_ee[q]))
        return set_err(c, CF_EINVAL, "init: non-finite H_ee / M_ee");

    // enriched cells in cell order, and grouped by colour for the setup scatter
    std::vector<int32_t> elist;
    std::vector<std::vector<int32_t>> ebycol(ncol);
    for (int64_t e = 0; e < E; ++e)
      if (ep[e + 1] > ep[e]) {
        elist.push_back((int32_t)e);
        ebycol[colour[e]].push_back((int32_t)e);
      }
    c->necells = (int)elist.size();

    // transposed per-cell blocks [NPAD][nap], nap = count padded to 16
    std::vector<int64_t> toff(E, 0);
    std::vector<int32_t> tld(E, 0);
    int64_t &ttot = c->ttot;
    for (int32_t e : elist) {
      const int na = (int)(ep[e + 1] - ep[e]);
      tld[e] = (na + 15) & ~15;
      toff[e] = ttot;
      ttot += (int64_t)NPAD * tld[e];
    }
    STCHK(dalloc(c, &c->HT, (size_t)std::max<int64_t>(ttot, 1)));
    STCHK(dalloc(c, &c->MT, (size_t)std::max<int64_t>(ttot, 1)));
    {
      std::vector<double> hb, mb;
      size_t ci0 = 0;
      while (ci0 < elist.size()) {
        // stage up to ~32 MB of blocks per copy
        size_t ci1 = ci0;
        int64_t len = 0;
        while (ci1 < elist.size() && (len == 0 || len + (int64_t)NPAD * tld[elist[ci1]] <= (4ll << 20))) {
          len += (int64_t)NPAD * tld[elist[ci1]];
          ++ci1;
        }
        hb.assign(len, 0.0);
        mb.assign(len, 0.0);
        const int64_t base = toff[elist[ci0]];
        for (size_t q = ci0; q < ci1; ++q) {
          const int32_t e = elist[q];
          const int nap = tld[e];
          double *ho = hb.data() + (toff[e] - base), *mo = mb.data() + (toff[e] - base);
          for (int64_t k = ep[e]; k < ep[e + 1]; ++k)
            for (int a = 0; a < npc; ++a) {
              ho[(int64_t)a * nap + (k - ep[e])] = pr->H_ec[k * npc + a];
              mo[(int64_t)a * nap + (k - ep[e])] = pr->M_ec[k * npc + a];
            }
        }
        HIPCHK(c, hipMemcpy(c->HT + base, hb.data(), len * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->MT + base, mb.data(), len * sizeof(double), hipMemcpyHostToDevice));
        ci0 = ci1;
      }
    }
    STCHK(dalloc(c, &c->toff, E));
    STCHK(dalloc(c, &c->tld, E));
    STCHK(dalloc(c, &c->eptr, E + 1));
    STCHK(dalloc(c, &c->ecells, std::max<size_t>(elist.size(), 1)));
    HIPCHK(c, hipMemcpy(c->toff, toff.data(), E * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->tld, tld.data(), E * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->eptr, ep, (E + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    if (!elist.empty())
      HIPCHK(c, hipMemcpy(c->ecells, elist.data(), elist.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    {
      std::vector<int32_t> perm(elist.size()), plist(elist.size());
      for (size_t q = 0; q < perm.size(); ++q) perm[q] = (int32_t)q;
      std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) {
        return ep[elist[x] + 1] - ep[elist[x]] > ep[elist[y] + 1] - ep[elist[y]];
      });
      for (size_t q = 0; q < perm.size(); ++q) plist[q] = elist[perm[q]];
      // items of the coupling partials: cells of 3 or more 16-row blocks take
      // one workgroup per group of 4 blocks.  Each cell (heaviest first) goes
      // to the least loaded of 8 queues, one per XCD (workgroup id mod 8), so
      // the groups of a cell gather their rows through one L2.
      {
        std::vector<std::vector<int32_t>> xq(8);
        std::vector<int64_t> xw(8, 0);
        for (size_t q = 0; q < plist.size(); ++q) {
          const int nmb = tld[plist[q]] >> 4;
          const int ng = nmb >= 3 ? (nmb + 3) / 4 : 1;
          const int x = (int)(std::min_element(xw.begin(), xw.end()) - xw.begin());
          for (int g = 0; g < ng; ++g) xq[x].push_back((int32_t)(q << 5) | g);
          xw[x] += nmb;
        }
        size_t len = 0;
        for (auto &v : xq) len = std::max(len, v.size());
        std::vector<int32_t> items(8 * len, -1);
        for (int x = 0; x < 8; ++x)
          for (size_t i = 0; i < xq[x].size(); ++i) items[8 * i + x] = xq[x][i];
        c->nepitems = (int)items.size();
        STCHK(dalloc(c, &c->epitems, std::max<size_t>(items.size(), 1)));
        if (!items.empty())
          HIPCHK(c, hipMemcpy(c->epitems, items.data(), items.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice));
      }
      STCHK(dalloc(c, &c->ecells_part, std::max<size_t>(plist.size(), 1)));
      STCHK(dalloc(c, &c->epos_part, std::max<size_t>(perm.size(), 1)));
      if (!plist.empty()) {
        HIPCHK(c, hipMemcpy(c->ecells_part, plist.data(), plist.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->epos_part, perm.data(), perm.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice));
      }
    }

    // alpha -> list of partial rows, increasing row index (fixed summation order)
    std::vector<int64_t> aptr(n_e + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) aptr[eidx[k] + 1]++;
    for (int64_t a = 0; a < n_e; ++a) aptr[a + 1] += aptr[a];
    std::vector<int32_t> alist(std::max<int64_t>(nnz, 1));
    {
      std::vector<int64_t> fill(aptr.begin(), aptr.end() - 1);
      for (int64_t k = 0; k < nnz; ++k) alist[fill[eidx[k]]++] = (int32_t)k;
    }
    STCHK(dalloc(c, &c->aptr, n_e + 1));
    STCHK(dalloc(c, &c->alist, alist.size()));
    HIPCHK(c, hipMemcpy(c->aptr, aptr.data(), (n_e + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->alist, alist.data(), alist.size() * sizeof(int32_t), hipMemcpyHostToDevice));

    // node-major coupling: CSR pattern over classical DOFs (columns = alpha)
    std::vector<int64_t> keys;
    for (int32_t e : elist)
      for (int a = 0; a < npc; ++a) {
        const int32_t d = dof[(int64_t)e * NPAD + a];
        if (d < 0) continue;
        for (int64_t k = ep[e]; k < ep[e + 1]; ++k) keys.push_back((int64_t)d * n_e + eidx[k]);
      }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    if ((int64_t)keys.size() >= (int64_t)INT32_MAX)
      return set_err(c, CF_EINVAL, "init: coupling pattern too large");
    c->csr_nnz = (int64_t)keys.size();
    std::vector<int32_t> rowptr(n_h + 1, 0), ci(std::max<size_t>(keys.size(), 1));
    for (size_t q = 0; q < keys.size(); ++q) {
      rowptr[keys[q] / n_e + 1]++;
      ci[q] = (int32_t)(keys[q] % n_e);
    }
    for (int64_t d = 0; d < n_h; ++d) rowptr[d + 1] += rowptr[d];
    std::vector<int32_t> smap((size_t)std::max<int64_t>(nnz, 1) * NPAD, -1);
    for (int32_t e : elist)
      for (int a = 0; a < npc; ++a) {
        const int32_t d = dof[(int64_t)e * NPAD + a];
        if (d < 0) continue;
        const int64_t *row = keys.data();
        for (int64_t k = ep[e]; k < ep[e + 1]; ++k) {
          const int64_t key = (int64_t)d * n_e + eidx[k];
          const int64_t pos = std::lower_bound(row + rowptr[d], row + rowptr[d + 1], key) - row;
          smap[k * NPAD + a] = (int32_t)pos;
        }
      }
    std::vector<int32_t> regrow;
    for (int64_t d = 0; d < n_h; ++d)
      if (rowptr[d + 1] > rowptr[d]) regrow.push_back((int32_t)d);
    const int64_t nreg = (int64_t)regrow.size();
    c->nreg = nreg;
    // classical DOF -> rows 128 e' + a of the enriched-cell buffer
    {
      std::vector<int32_t> qptr(n_h + 1, 0);
      for (size_t q = 0; q < elist.size(); ++q)
        for (int a = 0; a < npc; ++a) {
          const int32_t d = dof[(int64_t)elist[q] * NPAD + a];
          if (d >= 0) qptr[d + 1]++;
        }
      for (int64_t d = 0; d < n_h; ++d) c->qmax = std::max(c->qmax, qptr[d + 1]);
      for (int64_t d = 0; d < n_h; ++d) qptr[d + 1] += qptr[d];
      std::vector<int32_t> qidx(std::max<int32_t>(qptr[n_h], 1));
      std::vector<int32_t> fill(qptr.begin(), qptr.end() - 1);
      for (size_t q = 0; q < elist.size(); ++q)
        for (int a = 0; a < npc; ++a) {
          const int32_t d = dof[(int64_t)elist[q] * NPAD + a];
          if (d >= 0) qidx[fill[d]++] = (int32_t)(q * NPAD + a);
        }
      STCHK(dalloc(c, &c->qptr, n_h + 1));
      STCHK(dalloc(c, &c->qidx, qidx.size()));
      HIPCHK(c, hipMemcpy(c->qptr, qptr.data(), (n_h + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
      HIPCHK(c, hipMemcpy(c->qidx, qidx.data(), qidx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    STCHK(dalloc(c, &c->Q, (size_t)std::max<int>(c->necells, 1) * NPAD * lw));
    // per-cell coupling rows padded to NPAD, kept for the transposed products
    STCHK(dalloc(c, &c->Hec, (size_t)std::max<int64_t>(nnz, 1) * NPAD));
    STCHK(dalloc(c, &c->Mec, (size_t)std::max<int64_t>(nnz, 1) * NPAD));
    STCHK(dalloc(c, &c->eidx, std::max<int64_t>(nnz, 1)));
    HIPCHK(c, hipMemcpy(c->eidx, eidx.data(), std::max<int64_t>(nnz, 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    {
      const int64_t batch = 4096;
      std::vector<double> hb((size_t)batch * NPAD), mb2((size_t)batch * NPAD);
      for (int64_t k0 = 0; k0 < nnz; k0 += batch) {
        const int64_t nbk = std::min(batch, nnz - k0);
        std::fill(hb.begin(), hb.end(), 0.0);
        std::fill(mb2.begin(), mb2.end(), 0.0);
        for (int64_t k = 0; k < nbk; ++k)
          for (int a = 0; a < npc; ++a) {
            hb[k * NPAD + a] = pr->H_ec[(k0 + k) * npc + a];
            mb2[k * NPAD + a] = pr->M_ec[(k0 + k) * npc + a];
          }
        HIPCHK(c, hipMemcpy(c->Hec + k0 * NPAD, hb.data(), nbk * NPAD * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->Mec + k0 * NPAD, mb2.data(), nbk * NPAD * sizeof(double), hipMemcpyHostToDevice));
      }
    }

    STCHK(dalloc(c, &c->Hee, n_e * n_e));
    STCHK(dalloc(c, &c->Mee, n_e * n_e));
    STCHK(dalloc(c, &c->Sinv, n_e * n_e));
    STCHK(dalloc(c, &c->Hmod, n_e * n_e));
    HIPCHK(c, hipMemcpy(c->Hee, pr->H_ee, n_e * n_e * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->Mee, pr->M_ee, n_e * n_e * sizeof(double), hipMemcpyHostToDevice));
    STCHK(dalloc(c, &c->P, (size_t)std::max<int64_t>(nnz, 1) * lw));
    STCHK(dalloc(c, &c->Wb, (size_t)n_e * lw));
    STCHK(dalloc(c, &c->Zb, (size_t)n_e * lw));

    // ---- setup on the device (temporaries released at the end):
    //  CSR values (assembly of the per-cell coupling blocks by colour),
    //  S = M^ee - M^ec D^-1 M^ec^T (Sec. IV.D), its Cholesky factor and S^-1,
    //  K = M^ec D^-1 H^ec^T and H^ee - K.
    std::vector<void *> temps;
    auto tmp_alloc = [&](void **p, size_t bytes) -> cf_status {
      *p = nullptr;
      if (hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(c, CF_ENOMEM, "init: temporary allocation of " + std::to_string(bytes) + " bytes failed");
      }
      temps.push_back(*p);
      return CF_OK;
    };
    auto tmp_free = [&]() { for (void *q : temps) (void)hipFree(q); temps.clear(); };
    cf_status st = CF_OK;
    do {
      double *BM = nullptr, *BH = nullptr, *Gt = nullptr, *Sw = nullptr, *GpS = nullptr,
             *svS = nullptr, *WS = nullptr, *WST = nullptr, *hv = nullptr, *mv = nullptr;
      int32_t *dsmap = nullptr, *dcol = nullptr, *dreg = nullptr, *drow = nullptr, *dci = nullptr;
      const size_t nb = (size_t)std::max<int64_t>(nnz, 1) * NPAD;
      int nchS;
      {
        const int64_t cap = (int64_t)(512ll << 20) / (8 * n_e * n_e);
        nchS = (int)std::max<int64_t>(8, std::min<int64_t>(256, cap) / 8 * 8);
      }
      if ((st = tmp_alloc((void **)&dsmap, nb * sizeof(int32_t))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&dcol, std::max<size_t>(elist.size(), 1) * sizeof(int32_t))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&dreg, std::max<int64_t>(nreg, 1) * sizeof(int32_t))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&drow, (n_h + 1) * sizeof(int32_t))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&dci, ci.size() * sizeof(int32_t))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&hv, ci.size() * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&mv, ci.size() * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&BM, (size_t)std::max<int64_t>(nreg, 1) * n_e * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&BH, (size_t)std::max<int64_t>(nreg, 1) * n_e * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&Gt, (size_t)n_e * n_e * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&Sw, (size_t)n_e * n_e * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&GpS, (size_t)nchS * n_e * n_e * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&svS, (size_t)n_e * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&WS, (size_t)n_e * n_e * sizeof(double))) != CF_OK) break;
      if ((st = tmp_alloc((void **)&WST, (size_t)n_e * n_e * sizeof(double))) != CF_OK) break;
      hipError_t he = hipSuccess;
#define SCH(call) if ((he = (call)) != hipSuccess) { st = set_err(c, CF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(he)); break; }
      SCH(hipMemcpy(drow, rowptr.data(), (n_h + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
      SCH(hipMemcpy(dci, ci.data(), ci.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      SCH(hipMemsetAsync(hv, 0, ci.size() * sizeof(double), c->stream));
      SCH(hipMemsetAsync(mv, 0, ci.size() * sizeof(double), c->stream));
      SCH(hipMemcpy(dsmap, smap.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice));
      {
        std::vector<int32_t> cat;
        std::vector<int> off(1, 0);
        for (int col = 0; col < ncol; ++col) {
          cat.insert(cat.end(), ebycol[col].begin(), ebycol[col].end());
          off.push_back((int)cat.size());
        }
        if (!cat.empty()) SCH(hipMemcpy(dcol, cat.data(), cat.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        for (int col = 0; col < ncol && he == hipSuccess; ++col)
          he = launch_csr_fill(c->stream, c->Hec, c->Mec, c->eptr, dsmap, dcol + off[col],
                               off[col + 1] - off[col], hv, mv);
        if (he != hipSuccess) { st = set_err(c, CF_EDEVICE, std::string("csr_fill: ") + hipGetErrorString(he)); break; }
      }
      if (nreg) SCH(hipMemcpy(dreg, regrow.data(), nreg * sizeof(int32_t), hipMemcpyHostToDevice));
      SCH(hipMemsetAsync(BM, 0, (size_t)std::max<int64_t>(nreg, 1) * n_e * sizeof(double), c->stream));
      SCH(hipMemsetAsync(BH, 0, (size_t)std::max<int64_t>(nreg, 1) * n_e * sizeof(double), c->stream));
      SCH(launch_csr_dense(c->stream, nreg, dreg, drow, dci, hv, mv, c->dinv, BM, BH, n_e));
      const int64_t crow = (std::max<int64_t>(nreg, 1) + nchS - 1) / nchS;
      // S = M^ee - (D^-1/2 M^ec^T)^T (D^-1/2 M^ec^T)
      SCH(launch_gram_partial(c->stream, BM, n_e, BM, n_e, nreg, (int)n_e, (int)n_e, nchS, crow, GpS,
                              GRAM_UPPER));
      SCH(launch_gram_reduce(c->stream, GpS, nchS, (int)n_e, (int)n_e, Gt, n_e, GRAM_UPPER));
      SCH(launch_sub(c->stream, n_e * n_e, c->Mee, Gt, Sw));
      SCH(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
      SCH(launch_cholesky(c->stream, Sw, (int)n_e, 0, 0.0, svS, c->flag));
      int h_flag = 0;
      SCH(hipMemcpyAsync(&h_flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      SCH(hipStreamSynchronize(c->stream));
      if (h_flag) {
        st = set_err(c, CF_ENOTSPD, "init: Schur complement not positive definite (pivot " +
                                        std::to_string(h_flag - 1) + ")");
        break;
      }
      SCH(launch_tri_inv_T(c->stream, Sw, svS, (int)n_e, WS));          // WS = L^-T
      SCH(launch_transpose(c->stream, (int)n_e, WS, n_e, WST));         // WST = L^-1
      SCH(launch_small_gemm(c->stream, (int)n_e, (int)n_e, (int)n_e, WS, n_e, WST, n_e, c->Sinv, n_e));
      // K = M^ec D^-1 H^ec^T, H^ee - K
      SCH(launch_gram_partial(c->stream, BM, n_e, BH, n_e, nreg, (int)n_e, (int)n_e, nchS, crow, GpS,
                              GRAM_FULL));
      SCH(launch_gram_reduce(c->stream, GpS, nchS, (int)n_e, (int)n_e, Gt, n_e, GRAM_FULL));
      SCH(launch_sub(c->stream, n_e * n_e, c->Hee, Gt, c->Hmod));
      SCH(hipStreamSynchronize(c->stream));
#undef SCH
    } while (0);
    (void)hipStreamSynchronize(c->stream);
    tmp_free();
    if (st != CF_OK) return st;
  }
  c->cell_enriched.assign(E, 0);
  if (n_e > 0)
    for (int64_t e = 0; e < E; ++e) c->cell_enriched[e] = pr->enr_ptr[e + 1] > pr->enr_ptr[e];
  // cell flags: first touch; last touch of a DOF no enriched cell contains
  {
    std::vector<uint8_t> inreg(n_h, 0);
    if (n_e > 0)
      for (int64_t e = 0; e < E; ++e)
        if (pr->enr_ptr[e + 1] > pr->enr_ptr[e])
          for (int a = 0; a < npc; ++a) {
            const int32_t d = dof[e * NPAD + a];
            if (d >= 0) inreg[d] = 1;
          }
    std::vector<uint8_t> flag(first.size(), 0);
    for (size_t q = 0; q < first.size(); ++q) flag[q] = first[q] ? CELL_FIRST : 0;
    std::vector<int32_t> rows;
    for (int64_t d = 0; d < n_h; ++d) {
      if (inreg[d]) rows.push_back((int32_t)d);
      else flag[last_slot[d]] |= CELL_FINISH;
    }
    HIPCHK(c, hipMemcpy(c->flagp, flag.data(), flag.size(), hipMemcpyHostToDevice));
    // per colour: cells with a DOF in the enriched region first
    std::vector<int32_t> split;
    split.reserve(order.size());
    c->near_cnt.assign(c->col_off.size() - 1, 0);
    for (size_t k = 0; k + 1 < c->col_off.size(); ++k) {
      std::vector<int32_t> far;
      for (int q = c->col_off[k]; q < c->col_off[k + 1]; ++q) {
        const int32_t e = order[q];
        bool near = false;
        for (int a = 0; a < npc && !near; ++a) {
          const int32_t d = dof[(int64_t)e * NPAD + a];
          near = d >= 0 && inreg[d];
        }
        if (near) { split.push_back(e); ++c->near_cnt[k]; }
        else far.push_back(e);
      }
      split.insert(split.end(), far.begin(), far.end());
    }
    STCHK(dalloc(c, &c->cells_split, split.size()));
    HIPCHK(c, hipMemcpy(c->cells_split, split.data(), split.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice));
    c->nregrows = (int64_t)rows.size();
    STCHK(dalloc(c, &c->regrows, std::max<size_t>(rows.size(), 1)));
    if (!rows.empty())
      HIPCHK(c, hipMemcpy(c->regrows, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CF_OK;
}

// ---------------------------------------------------------------------------
// batches of independent problems
// ---------------------------------------------------------------------------
// Entries that point to the same cf_problem share one context (its device
// operator, and its FP64 workspace for the per-entry Rayleigh-Ritz and
// Lanczos calls, which run one after another); every entry has its own FP32
// recurrence workspace, so the batched filter runs all entries at once.
struct cf_batch {
  int device = 0;
  hipStream_t caller = nullptr, bs = nullptr;
  int count = 0;
  int64_t max_cols = 0;
  std::vector<cf_ctx *> uniq;
  std::vector<int> which;                   // entry -> uniq index
  // device descriptors and work lists
  std::vector<BatchProb> h_bp;
  BatchProb *stage = nullptr;               // pinned staging of the per-call descriptors
  BatchProb *d_bp = nullptr;
  std::vector<int> cell_off_all, cell_off_near, cell_off_far;   // per colour, into d_items
  BatchItem *d_items = nullptr;
  BatchItem *d_eitems = nullptr;
  int neitems = 0, kmax = 0, ncolours = 0, lp_cap = 0;
  int64_t *d_boff = nullptr, *d_aoff = nullptr, *d_eoff = nullptr;
  int64_t nbblocks = 0, nalpha = 0, neblocks = 0;
  bool lowp_ready = false, bf16_ready = false;
  // graph of the batched filter, keyed by (m, prec)
  hipGraphExec_t gexec = nullptr;
  int g_m = -1, g_prec = -1, g_nsb = -1;
  // column blocks per tile of the batched reduced cell product, FP32-input
  // cells [0] and BF16-input cells [1] (chebfilter_batch_autotune)
  int nsb[2] = {1, 2};
  int bmap = CPL_BMAP_DEFAULT;              // coupling-partials split by row-block bucket
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_copy = nullptr;
  bool copy_pending = false;
  // batched projection and Lanczos (allocated on first use): per-entry status
  // words (8 each), projected pencils, Ritz values and eigensolver info by
  // slot (entries sorted by block width), the entry -> slot map, the bounds
  int *d_rst = nullptr, *d_rinfo = nullptr, *d_rslot = nullptr;
  double *d_rH = nullptr, *d_rM = nullptr, *d_rth = nullptr, *d_rE = nullptr, *d_lz = nullptr;
  std::vector<int> h_rslot, h_rst;
  std::vector<double> h_rth, h_lz;
  // Lanczos runs of entries that share a problem go together as the columns
  // of one block (at most max_cols per group): groups, workspace blocks
  std::vector<std::vector<int>> lz_groups;
  double *d_lzblk = nullptr, *d_lzc = nullptr, *d_lzp = nullptr;
  int64_t lz_n = 0;
  int lz_k = 0;
  std::string err;
  std::vector<void *> allocs;
};

static cf_status berr(cf_batch *b, cf_status st, const std::string &msg) {
  if (b) b->err = msg; else g_init_error = msg;
  return st;
}

#define BHIPCHK(b, call)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return berr(b, CF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

template <typename T>
static cf_status balloc(cf_batch *b, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void *q = nullptr;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return berr(b, CF_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  b->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return CF_OK;
}

template <typename T>
static cf_status bupload(cf_batch *b, T **p, const std::vector<T> &v) {
  cf_status st = balloc(b, p, v.size());
  if (st != CF_OK) return st;
  if (!v.empty()) BHIPCHK(b, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return CF_OK;
}

static void free_batch(cf_batch *b) {
  if (!b) return;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  for (cf_ctx *c : b->uniq) free_ctx(c);
  for (void *q : b->allocs) (void)hipFree(q);
  if (b->stage) (void)hipHostFree(b->stage);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->ev_copy) (void)hipEventDestroy(b->ev_copy);
  if (b->bs) (void)hipStreamDestroy(b->bs);
  delete b;
}

// Reduced-precision operator copies of every problem, FP32 workspace of every
// entry, descriptors and work lists (once; BF16 copies on first BF16 use).
static cf_status batch_prepare_lowp(cf_batch *b, bool bf16, int m) {
  for (cf_ctx *c : b->uniq) {
    cf_status st = ensure_lowp(c, bf16);
    if (st != CF_OK) return berr(b, st, c->err);
  }
  if (bf16) b->bf16_ready = true;
  const int cap = std::max(256, m + 2);
  const bool new_cap = cap > b->lp_cap;
  if (b->lowp_ready && !new_cap) {
    if (bf16)
      for (int i = 0; i < b->count; ++i) b->h_bp[i].Hp16 = b->uniq[b->which[i]]->Hp16;
    return CF_OK;
  }
  const int64_t mc = b->max_cols;
  if (!b->lowp_ready) b->h_bp.assign(b->count, BatchProb());
  for (int i = 0; i < b->count; ++i) {
    cf_ctx *c = b->uniq[b->which[i]];
    BatchProb &P = b->h_bp[i];
    P.Hp32 = c->Hp32; P.Hp16 = c->Hp16; P.dofp = c->dofp; P.flagp = c->flagp;
    P.HT32 = c->HT32; P.MT32 = c->MT32; P.toff = c->toff; P.tld = c->tld; P.eptr = c->eptr;
    P.ecells = c->ecells; P.Hec32 = c->Hec32; P.Mec32 = c->Mec32; P.eidx = c->eidx;
    P.aptr = c->aptr; P.alist = c->alist; P.Hmod = c->Hmod; P.Sinv = c->Sinv; P.dinv = c->dinv;
    P.qptr = c->qptr; P.qidx = c->qidx; P.regrows = c->regrows;
    P.nregrows = c->nregrows; P.n_h = c->n_h; P.n_e = c->n_e; P.n = c->n;
    P.mc = mc;
    if (!b->lowp_ready) {
      STCHK(balloc(b, &P.F0, (size_t)c->n * mc));
      STCHK(balloc(b, &P.F1, (size_t)c->n * mc));
      STCHK(balloc(b, &P.R32, (size_t)c->n_h * mc));
      if (c->n_e > 0) {
        STCHK(balloc(b, &P.P32, (size_t)std::max<int64_t>(c->nnz, 1) * mc));
        STCHK(balloc(b, &P.Q32, (size_t)std::max<int>(c->necells, 1) * NPAD * mc));
        STCHK(balloc(b, &P.Wb, (size_t)c->n_e * mc));
        STCHK(balloc(b, &P.Zb, (size_t)c->n_e * mc));
      }
    }
    if (new_cap) {
      STCHK(balloc(b, &P.lp_mx, (size_t)cap * MX_SLOTS));
      STCHK(balloc(b, &P.lp_s, (size_t)cap));
      STCHK(balloc(b, &P.lp_mult, (size_t)2 * cap));
    }
  }
  b->lp_cap = std::max(b->lp_cap, cap);
  if (!b->lowp_ready) {
    STCHK(balloc(b, &b->d_bp, (size_t)b->count));
    if (hipHostMalloc((void **)&b->stage, (size_t)b->count * sizeof(BatchProb)) != hipSuccess)
      return berr(b, CF_ENOMEM, "hipHostMalloc of the descriptor staging failed");
    // work lists: per colour all cells / near cells / far cells of every entry
    std::vector<BatchItem> items;
    b->ncolours = 0;
    for (cf_ctx *c : b->uniq) b->ncolours = std::max(b->ncolours, (int)c->col_off.size() - 1);
    std::vector<std::vector<int32_t>> split(b->uniq.size());
    for (size_t u = 0; u < b->uniq.size(); ++u) {
      cf_ctx *c = b->uniq[u];
      split[u].resize(c->col_off.back());
      BHIPCHK(b, hipMemcpy(split[u].data(), c->cells_split, split[u].size() * sizeof(int32_t),
                           hipMemcpyDeviceToHost));
    }
    b->cell_off_all.assign(b->ncolours + 1, 0);
    b->cell_off_near.assign(b->ncolours + 1, 0);
    b->cell_off_far.assign(b->ncolours + 1, 0);
    auto add = [&](int k, int part) {
      for (int i = 0; i < b->count; ++i) {
        const int u = b->which[i];
        cf_ctx *c = b->uniq[u];
        if (k + 1 >= (int)c->col_off.size()) continue;
        const int c0 = c->col_off[k], cnt = c->col_off[k + 1] - c0, nn = c->near_cnt[k];
        const int q0 = part == 2 ? c0 + nn : c0;
        const int q1 = part == 1 ? c0 + nn : c0 + cnt;
        for (int q = q0; q < q1; ++q) items.push_back({i, split[u][q]});
      }
    };
    for (int k = 0; k < b->ncolours; ++k) {          // all cells (FP32 form)
      b->cell_off_all[k] = (int)items.size();
      add(k, 0);
    }
    b->cell_off_all[b->ncolours] = (int)items.size();
    for (int k = 0; k < b->ncolours; ++k) {          // near cells (FP32 in the BF16 form)
      b->cell_off_near[k] = (int)items.size();
      add(k, 1);
    }
    b->cell_off_near[b->ncolours] = (int)items.size();
    for (int k = 0; k < b->ncolours; ++k) {          // far cells (BF16)
      b->cell_off_far[k] = (int)items.size();
      add(k, 2);
    }
    b->cell_off_far[b->ncolours] = (int)items.size();
    STCHK(bupload(b, &b->d_items, items));
    std::vector<BatchItem> eitems;
    std::vector<int64_t> boff(1, 0), aoff(1, 0), eoff(1, 0);
    b->kmax = 0;
    for (int i = 0; i < b->count; ++i) {
      cf_ctx *c = b->uniq[b->which[i]];
      for (int j = 0; j < c->necells; ++j) eitems.push_back({i, j});
      b->kmax = std::max(b->kmax, c->kmax);
      boff.push_back(boff.back() + std::max<int64_t>((c->n + 63) / 64, 1));
      aoff.push_back(aoff.back() + c->n_e);
      eoff.push_back(eoff.back() + std::max<int64_t>((c->nregrows + c->n_e + 15) / 16, 1));
    }
    b->neitems = (int)eitems.size();
    b->nbblocks = boff.back();
    b->nalpha = aoff.back();
    b->neblocks = eoff.back();
    STCHK(bupload(b, &b->d_eitems, eitems));
    STCHK(bupload(b, &b->d_boff, boff));
    STCHK(bupload(b, &b->d_aoff, aoff));
    STCHK(bupload(b, &b->d_eoff, eoff));
    BHIPCHK(b, prepare_b_enr(b->kmax));
    b->lowp_ready = true;
  }
  if (new_cap && b->gexec) {           // descriptors of the captured graph moved
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  return CF_OK;
}

// The batched filter's launches (steps 0..m-1), enqueued on b->bs.
static cf_status batch_enqueue_filter(cf_batch *b, int m, bool bf16) {
  hipStream_t s = b->bs;
  BHIPCHK(b, launch_b_lp_begin(s, b->d_bp, b->count, (m + 2) * MX_SLOTS, b->d_boff, b->nbblocks));
  for (int k = 0; k < m; ++k) {
    if (k > 0) BHIPCHK(b, launch_b_lp_scale(s, b->d_bp, b->count, k));
    for (int col = 0; col < b->ncolours; ++col) {
      if (bf16) {
        const int n0 = b->cell_off_near[col], n1 = b->cell_off_near[col + 1];
        const int f0 = b->cell_off_far[col], f1 = b->cell_off_far[col + 1];
        BHIPCHK(b, launch_b_cell(s, false, b->nsb[0], b->d_bp, b->d_items + n0, n1 - n0, k));
        BHIPCHK(b, launch_b_cell(s, true, b->nsb[1], b->d_bp, b->d_items + f0, f1 - f0, k));
      } else {
        const int a0 = b->cell_off_all[col], a1 = b->cell_off_all[col + 1];
        BHIPCHK(b, launch_b_cell(s, false, b->nsb[0], b->d_bp, b->d_items + a0, a1 - a0, k));
      }
    }
    BHIPCHK(b, launch_b_enr(s, b->d_bp, b->count, b->d_eitems, b->neitems, b->d_aoff, b->nalpha,
                            (int)b->max_cols, b->kmax, k, b->bmap));
    BHIPCHK(b, launch_b_epilogue(s, b->d_bp, b->count, b->d_eoff, b->neblocks, k));
  }
  BHIPCHK(b, launch_b_lp_output(s, b->d_bp, b->count, b->d_boff, b->nbblocks, m));
  return CF_OK;
}

// ---------------------------------------------------------------------------
// public entry points
// ---------------------------------------------------------------------------
extern "C" {

cf_status chebfilter_init(const cf_problem *prob, const cf_options *opt, cf_ctx **out) {
  if (!out) return set_err(nullptr, CF_EINVAL, "init: null output pointer");
  *out = nullptr;
  cf_ctx *c = new (std::nothrow) cf_ctx();
  if (!c) return set_err(nullptr, CF_ENOMEM, "init: host allocation failed");
  cf_status st = do_init(prob, opt, c);
  if (st != CF_OK) {
    g_init_error = c->err;
    free_ctx(c);
    return st;
  }
  *out = c;
  return CF_OK;
}

cf_status chebfilter_destroy(cf_ctx *ctx) {
  if (!ctx) return CF_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
  return CF_OK;
}

const char *chebfilter_last_error(const cf_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

cf_status chebfilter_sizes(const cf_ctx *ctx, int64_t *n_h, int64_t *n_e, int64_t *max_cols) {
  if (!ctx) return CF_EINVAL;
  if (n_h) *n_h = ctx->n_h;
  if (n_e) *n_e = ctx->n_e;
  if (max_cols) *max_cols = ctx->max_cols;
  return CF_OK;
}

cf_status chebfilter_apply_H(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                             int64_t N) {
  if (!c) return CF_EINVAL;
  STCHK(check_block(c, X, ldx, N, "apply_H X"));
  STCHK(check_block(c, Y, ldy, N, "apply_H Y"));
  if (N == 0) return CF_OK;
  HIPCHK(c, hipSetDevice(c->device));
  for (int64_t j0 = 0; j0 < N; j0 += c->chunk)
    STCHK(core_apply_H(c, X + j0, ldx, Y + j0, ldy, (int)std::min(c->chunk, N - j0)));
  return CF_OK;
}

cf_status chebfilter_apply_M(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                             int64_t N) {
  if (!c) return CF_EINVAL;
  STCHK(check_block(c, X, ldx, N, "apply_M X"));
  STCHK(check_block(c, Y, ldy, N, "apply_M Y"));
  if (N == 0) return CF_OK;
  HIPCHK(c, hipSetDevice(c->device));
  for (int64_t j0 = 0; j0 < N; j0 += c->chunk)
    STCHK(core_apply_M(c, X + j0, ldx, Y + j0, ldy, (int)std::min(c->chunk, N - j0)));
  return CF_OK;
}

cf_status chebfilter_apply_Sinv(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                                int64_t N) {
  if (!c) return CF_EINVAL;
  STCHK(check_block(c, X, ldx, N, "apply_Sinv X"));
  STCHK(check_block(c, Y, ldy, N, "apply_Sinv Y"));
  if (N == 0) return CF_OK;
  HIPCHK(c, hipSetDevice(c->device));
  for (int64_t j0 = 0; j0 < N; j0 += c->chunk)
    STCHK(core_apply_Sinv(c, X + j0, ldx, Y + j0, ldy, (int)std::min(c->chunk, N - j0)));
  return CF_OK;
}

// One column chunk (n <= ldw) of the filter; X must not be Y.
static cf_status core_filter_chunk(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                                   int n, int m, double e, double cc, int32_t prec) {
  if (prec != CF_FP64) {
    // FP32 recurrence: Y_k lives in F0 (k even) or F1 (k odd); Y_{k+1}
    // overwrites Y_{k-1} element by element
    // The iterates are held as Z_k = Y_k 2^-s_k with s_k chosen on the device
    // from the growth of the last two iterates (powers of two: every rounding
    // is that of the unscaled recurrence, which would leave FP32's range at
    // high degree or wide damping intervals); Y = Z_m 2^s_m is formed in FP64.
    const bool bf16 = prec == CF_BF16;
    STCHK(ensure_lowp(c, bf16));
    STCHK(ensure_lp_scale(c, m));
    const int64_t mc = c->ldw;
    float *F[2] = {c->F0, c->F1};
    HIPCHK(c, launch_lp_reset(c->stream, c->lp_mx, (m + 2) * MX_SLOTS));
    HIPCHK(c, launch_lp_input(c->stream, c->n, n, X, ldx, c->F0, mc, c->lp_mx));
    HIPCHK(c, launch_lp_scale(c->stream, 0, c->lp_mx, c->lp_s, c->lp_mult));
    STCHK(core_htilde_step_lp(c, bf16, F[0], mc, n, (float)e, (float)-cc, nullptr, 0, 0.f, F[1], mc,
                              c->lp_mult, c->lp_mx + MX_SLOTS));
    for (int k = 1; k < m; ++k) {
      HIPCHK(c, launch_lp_scale(c->stream, k, c->lp_mx, c->lp_s, c->lp_mult));
      STCHK(core_htilde_step_lp(c, bf16, F[k & 1], mc, n, (float)(2.0 * e), (float)(-2.0 * cc),
                                F[(k - 1) & 1], mc, -1.f, F[(k + 1) & 1], mc, c->lp_mult + 2 * k,
                                c->lp_mx + (k + 1) * MX_SLOTS));
    }
    HIPCHK(c, launch_lp_output(c->stream, c->n, n, F[m & 1], mc, c->lp_s + m, Y, ldy));
    return CF_OK;
  }
  // Y_k lives in Y when (m - k) is even, else in the internal block B2.
  auto buf = [&](int k) -> double * { return ((m - k) % 2 == 0) ? Y : c->B2; };
  auto ldb = [&](int k) -> int64_t { return ((m - k) % 2 == 0) ? ldy : c->ldw; };
  STCHK(core_htilde_step(c, X, ldx, n, e, X, ldx, -cc, nullptr, 0, 0.0, buf(1), ldb(1)));
  for (int k = 1; k < m; ++k) {
    const double *prev = (k == 1) ? X : buf(k - 1);
    const int64_t ldp = (k == 1) ? ldx : ldb(k - 1);
    STCHK(core_htilde_step(c, buf(k), ldb(k), n, 2.0 * e, buf(k), ldb(k), -2.0 * cc, prev, ldp, -1.0,
                           buf(k + 1), ldb(k + 1)));
  }
  return CF_OK;
}

cf_status chebfilter_filter(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                            int64_t N, int32_t m, double a, double b, int32_t prec) {
  if (!c) return CF_EINVAL;
  STCHK(check_block(c, X, ldx, N, "filter X"));
  STCHK(check_block(c, Y, ldy, N, "filter Y"));
  if (m < 0) return set_err(c, CF_EINVAL, "filter: m < 0");
  if (!std::isfinite(a) || !std::isfinite(b) || !(b > a))
    return set_err(c, CF_EINVAL, "filter: need finite a < b");
  if (prec != CF_FP64 && prec != CF_FP32 && prec != CF_BF16)
    return set_err(c, CF_EINVAL, "filter: prec must be CF_FP64, CF_FP32 or CF_BF16");
  if (N == 0) return CF_OK;
  const bool inplace = X == Y;
  if (inplace && ldx != ldy) return set_err(c, CF_EINVAL, "filter: in place needs ldx == ldy");
  HIPCHK(c, hipSetDevice(c->device));
  if (m == 0) {
    if (!inplace) HIPCHK(c, launch_copy(c->stream, c->n, (int)N, X, ldx, Y, ldy));
    return CF_OK;
  }
  // t(H~) = e H~ - cc I with e = 2/(b-a), cc = (a+b)/(b-a).  The columns are
  // independent: chunks of at most ldw columns run one after another.  In
  // place, an FP64 chunk is read from a copy in the work block U (the FP32
  // forms read it once into their own blocks before the chunk is written).
  const double e = 2.0 / (b - a), cc = (a + b) / (b - a);
  for (int64_t j0 = 0; j0 < N; j0 += c->chunk) {
    const int nc = (int)std::min(c->chunk, N - j0);
    const double *Xc = X + j0;
    int64_t ldxc = ldx;
    if (inplace && prec == CF_FP64) {
      HIPCHK(c, launch_copy(c->stream, c->n, nc, X + j0, ldx, c->U, c->ldw));
      Xc = c->U;
      ldxc = c->ldw;
    }
    STCHK(core_filter_chunk(c, Xc, ldxc, Y + j0, ldy, nc, m, e, cc, prec));
  }
  return check_out_finite(c, Y, ldy, (int)N, "filter");
}

cf_status chebfilter_filter_multipass(cf_ctx *c, const double *X, int64_t ldx, double *Y,
                                     int64_t ldy, int64_t N, int32_t m, int32_t passes, double a,
                                     double b, int32_t prec) {
  if (!c) return CF_EINVAL;
  if (passes < 1) return set_err(c, CF_EINVAL, "filter_multipass: passes must be >= 1");
  if (passes == 1) return chebfilter_filter(c, X, ldx, Y, ldy, N, m, a, b, prec);
  STCHK(check_block(c, X, ldx, N, "filter_multipass X"));
  STCHK(check_block(c, Y, ldy, N, "filter_multipass Y"));
  if (X == Y && ldx != ldy) return set_err(c, CF_EINVAL, "filter_multipass: in place needs ldx == ldy");
  if (N == 0) return CF_OK;
  HIPCHK(c, hipSetDevice(c->device));
  // every pass ends in Y; the next one filters Y in place
  std::vector<double> theta((size_t)N);
  STCHK(chebfilter_filter(c, X, ldx, Y, ldy, N, m, a, b, prec));
  for (int i = 1; i < passes; ++i) {
    // Rayleigh-Ritz between passes: the Ritz vectors keep each column aligned
    // with its own eigen-direction, so the next pass amplifies them one by
    // one (a triangular Cholesky-QR basis would mix them, and after a second
    // high-degree pass the columns would all lean towards the lowest one)
    STCHK(chebfilter_rayleigh_ritz(c, Y, ldy, N, theta.data()));
    STCHK(chebfilter_filter(c, Y, ldy, Y, ldy, N, m, a, b, prec));
  }
  return CF_OK;
}

cf_status chebfilter_cholqr(cf_ctx *c, double *Y, int64_t ldy, int64_t N) {
  if (!c) return CF_EINVAL;
  STCHK(check_block(c, Y, ldy, N, "cholqr Y"));
  if (N == 0) return CF_OK;
  HIPCHK(c, hipSetDevice(c->device));
  STCHK(core_cholqr(c, Y, ldy, Y, ldy, (int)N));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CF_OK;
}

cf_status chebfilter_rayleigh_ritz(cf_ctx *c, double *Y, int64_t ldy, int64_t N,
                                   double *theta_host) {
  if (!c) return CF_EINVAL;
  STCHK(check_block(c, Y, ldy, N, "rayleigh_ritz Y"));
  if (N > 0 && !theta_host) return set_err(c, CF_EINVAL, "rayleigh_ritz: null theta");
  if (N == 0) return CF_OK;
  HIPCHK(c, hipSetDevice(c->device));
  const int n = (int)N;
  const int64_t ld = c->ldw, cw = c->chunk;
  // Q (Euclidean-orthonormal): in U when the block fits the work blocks,
  // else in Y itself
  const bool wide = N > cw;
  double *Qb = wide ? Y : c->U;
  const int64_t ldq = wide ? ldy : ld;
  STCHK(core_cholqr(c, Y, ldy, Qb, ldq, n));
  // projected pencil
  if (!wide) {
    STCHK(core_apply_H(c, Qb, ldq, c->T, ld, n));
    STCHK(core_gram(c, Qb, ldq, c->T, ld, c->n, n, c->Hh, GRAM_SYM));
    STCHK(core_apply_M(c, Qb, ldq, c->T, ld, n));
    STCHK(core_gram(c, Qb, ldq, c->T, ld, c->n, n, c->Mh, GRAM_SYM));
  } else {
    // column chunk [j0, j1): T = H Q[:, j0:j1], then the slab rows 0..j1 of
    // Q^T T (the upper triangle and the chunk's diagonal block); likewise M;
    // the lower triangles are mirrored from the upper ones
    for (int64_t j0 = 0; j0 < N; j0 += cw) {
      const int nc = (int)std::min(cw, N - j0);
      const int j1 = (int)j0 + nc;
      STCHK(core_apply_H(c, Qb + j0, ldq, c->T, ld, nc));
      STCHK(core_gram_slab(c, Qb, ldq, j1, c->T, ld, nc, c->Hh + j0, n));
      STCHK(core_apply_M(c, Qb + j0, ldq, c->T, ld, nc));
      STCHK(core_gram_slab(c, Qb, ldq, j1, c->T, ld, nc, c->Mh + j0, n));
    }
    HIPCHK(c, launch_mirror_upper(c->stream, c->Hh, n));
    HIPCHK(c, launch_mirror_upper(c->stream, c->Mh, n));
  }
  // the projected pencil (Hh, Mh) to standard form: Mh = L L^T (library
  // Cholesky; on the row-major symmetric Mh the column-major upper factor is
  // the row-major lower L), W = L^-T, C = W^T Hh W; symmetric eigensolve of C;
  // Ritz vectors Y = Q (W V).  All row-major N x N products go to rocBLAS
  // through the column-major view (a row-major X is the column-major X^T).
  HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  if (rocsolver_dpotrf(c->rb, rocblas_fill_upper, n, c->Mh, n, (rocblas_int *)c->flag) !=
      rocblas_status_success)
    return set_err(c, CF_EDEVICE, "rayleigh_ritz: rocsolver_dpotrf failed");
  HIPCHK(c, launch_tri_inv_T(c->stream, c->Mh, nullptr, n, c->Wt));
  {
    const double one = 1.0, zero = 0.0;
    rocblas_set_pointer_mode(c->rb, rocblas_pointer_mode_host);
    // G = Hh W (row-major), then Hh <- W^T G
    if (rocblas_dgemm(c->rb, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, c->Wt,
                      n, c->Hh, n, &zero, c->G, n) != rocblas_status_success ||
        rocblas_dgemm(c->rb, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one,
                      c->G, n, c->Wt, n, &zero, c->Hh, n) != rocblas_status_success)
      return set_err(c, CF_EDEVICE, "rayleigh_ritz: rocblas_dgemm failed");
  }
  if (rocsolver_dsyevd(c->rb, rocblas_evect_original, rocblas_fill_upper, n, c->Hh, n, c->theta,
                       c->evE, c->info) != rocblas_status_success)
    return set_err(c, CF_EDEVICE, "rayleigh_ritz: rocsolver_dsyevd failed");
  {
    // Wm = W V (row-major); the eigenvectors are the columns of the
    // column-major V in Hh
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(c->rb, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &one,
                      c->Hh, n, c->Wt, n, &zero, c->Wm, n) != rocblas_status_success)
      return set_err(c, CF_EDEVICE, "rayleigh_ritz: rocblas_dgemm failed");
  }
  rocblas_int h_info = 0;
  int h_flag = 0;
  HIPCHK(c, hipMemcpyAsync(&h_info, c->info, sizeof(rocblas_int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&h_flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(theta_host, c->theta, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // a failed factorisation or eigensolve leaves the block as it was (the
  // orthonormal basis when it was formed in place)
  if (h_flag) return set_err(c, CF_ENOTSPD, "rayleigh_ritz: projected overlap not SPD");
  if (h_info > 0) return set_err(c, CF_ENOTCONV, "rayleigh_ritz: eigensolver did not converge");
  STCHK(core_rotate(c, Qb, ldq, c->Wm, n, Y, ldy));
  return check_out_finite(c, Y, ldy, n, "rayleigh_ritz");
}

cf_status chebfilter_lanczos_bounds(cf_ctx *c, const double *v0, int32_t k, double *lmin_est,
                                    double *b_upper) {
  if (!c) return CF_EINVAL;
  if (!v0 || !lmin_est || !b_upper) return set_err(c, CF_EINVAL, "lanczos: null argument");
  if (k < 1 || k > 64) return set_err(c, CF_EINVAL, "lanczos: k must be 1..64");
  HIPCHK(c, hipSetDevice(c->device));
  double *dout = c->lzcoef + 2 * 64 + 2;
  STCHK(core_lanczos(c, v0, k, dout));
  double out2[2] = {0.0, 0.0};
  HIPCHK(c, hipMemcpyAsync(out2, dout, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *lmin_est = out2[0];
  *b_upper = out2[1];
  if (!std::isfinite(out2[0]) || !std::isfinite(out2[1]))
    return set_err(c, CF_ENUMERIC, "lanczos: non-finite bound (breakdown?)");
  return CF_OK;
}

cf_status chebfilter_lanczos_bounds_noalloc(cf_ctx *c, const double *v0, int32_t k,
                                            double *lmin_est, double *b_upper) {
  if (!c) return CF_EINVAL;
  if (!v0 || !lmin_est || !b_upper) return set_err(c, CF_EINVAL, "lanczos_noalloc: null argument");
  if (k < 1 || k > 64) return set_err(c, CF_EINVAL, "lanczos_noalloc: k must be 1..64");
  const int64_t need = noalloc_need(c);
  if (need > NOALLOC_DOUBLES)
    return set_err(c, CF_ENOMEM, "lanczos_noalloc: the problem needs " +
                                     std::to_string(need * 8 / (1 << 20) + 1) +
                                     " MiB of scratch; the fixed scratch holds 64 MiB");
  HIPCHK(c, hipSetDevice(c->device));
  double *base = nullptr;
  STCHK(scratch_address(c, &base));
  double out2[2] = {0.0, 0.0};
  {
    ScratchWork sw(c, base);
    double *dout = c->lzcoef + 2 * 64 + 2;
    STCHK(core_lanczos(c, v0, k, dout));
    HIPCHK(c, hipMemcpyAsync(out2, dout, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  *lmin_est = out2[0];
  *b_upper = out2[1];
  if (!std::isfinite(out2[0]) || !std::isfinite(out2[1]))
    return set_err(c, CF_ENUMERIC, "lanczos_noalloc: non-finite bound (breakdown?)");
  return CF_OK;
}

cf_status chebfilter_profile(cf_ctx *c, int32_t enable) {
  if (!c) return CF_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto &kv : c->prof)
    for (auto &ev : kv.second.pending) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  c->prof.clear();
  c->profiling = enable != 0;
  return CF_OK;
}

cf_status chebfilter_profile_query(cf_ctx *c, const char *name, int64_t *launches,
                                   double *total_ms, double *total_flops) {
  if (!c || !name) return CF_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  auto it = c->prof.find(name);
  if (it == c->prof.end()) {
    if (launches) *launches = 0;
    if (total_ms) *total_ms = 0.0;
    if (total_flops) *total_flops = 0.0;
    return CF_OK;
  }
  ProfEntry &pe = it->second;
  for (auto &ev : pe.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) pe.ms += ms;
    pe.launches += 1;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  pe.pending.clear();
  if (launches) *launches = pe.launches;
  if (total_ms) *total_ms = pe.ms;
  if (total_flops) *total_flops = pe.flops;
  return CF_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
cf_status chebfilter_init_batch(const cf_problem *const *probs, int32_t count, const cf_options *opt,
                                cf_batch **out) {
  if (!out) return berr(nullptr, CF_EINVAL, "init_batch: null output pointer");
  *out = nullptr;
  if (!probs || count < 1 || !opt) return berr(nullptr, CF_EINVAL, "init_batch: need count >= 1 problems");
  cf_batch *b = new (std::nothrow) cf_batch();
  if (!b) return berr(nullptr, CF_ENOMEM, "init_batch: host allocation failed");
  b->device = opt->device;
  b->caller = (hipStream_t)opt->stream;
  b->count = count;
  b->max_cols = opt->max_cols;
  // the batched kernels take each block whole: no column chunks
  cf_options ob = *opt;
  ob.col_chunk = 0;
  std::map<const cf_problem *, int> seen;
  for (int i = 0; i < count; ++i) {
    if (!probs[i]) { free_batch(b); return berr(nullptr, CF_EINVAL, "init_batch: null problem"); }
    auto it = seen.find(probs[i]);
    if (it != seen.end()) { b->which.push_back(it->second); continue; }
    cf_ctx *c = new (std::nothrow) cf_ctx();
    if (!c) { free_batch(b); return berr(nullptr, CF_ENOMEM, "init_batch: host allocation failed"); }
    cf_status st = do_init(probs[i], &ob, c);
    if (st != CF_OK) {
      g_init_error = "init_batch: problem " + std::to_string(i) + ": " + c->err;
      free_ctx(c);
      free_batch(b);
      return st;
    }
    seen[probs[i]] = (int)b->uniq.size();
    b->which.push_back((int)b->uniq.size());
    b->uniq.push_back(c);
  }
  if (hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_copy, hipEventDisableTiming) != hipSuccess) {
    free_batch(b);
    return berr(nullptr, CF_EDEVICE, "init_batch: stream or event creation failed");
  }
  *out = b;
  return CF_OK;
}

cf_status chebfilter_batch_destroy(cf_batch *b) {
  if (!b) return CF_OK;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->bs);
  (void)hipStreamSynchronize(b->caller);
  free_batch(b);
  return CF_OK;
}

const char *chebfilter_batch_last_error(const cf_batch *b) {
  return b ? b->err.c_str() : g_init_error.c_str();
}

cf_status chebfilter_batch_sizes(const cf_batch *b, int32_t i, int64_t *n_h, int64_t *n_e) {
  if (!b || i < 0 || i >= b->count) return CF_EINVAL;
  const cf_ctx *c = b->uniq[b->which[i]];
  if (n_h) *n_h = c->n_h;
  if (n_e) *n_e = c->n_e;
  return CF_OK;
}

cf_status chebfilter_filter_batch(cf_batch *b, const double *const *X, const int64_t *ldx,
                                  double *const *Y, const int64_t *ldy, const int64_t *N, int32_t m,
                                  const double *a, const double *bu, int32_t prec, int32_t use_graph) {
  if (!b) return CF_EINVAL;
  if (!X || !ldx || !Y || !ldy || !N || !a || !bu)
    return berr(b, CF_EINVAL, "filter_batch: null argument array");
  if (m < 0) return berr(b, CF_EINVAL, "filter_batch: m < 0");
  if (prec != CF_FP64 && prec != CF_FP32 && prec != CF_BF16)
    return berr(b, CF_EINVAL, "filter_batch: prec must be CF_FP64, CF_FP32 or CF_BF16");
  for (int i = 0; i < b->count; ++i) {
    if (N[i] < 1 || N[i] > b->max_cols)
      return berr(b, N[i] < 1 ? CF_EINVAL : CF_ENOMEM, "filter_batch: N[" + std::to_string(i) +
                                                           "] out of range [1, max_cols]");
    if (!X[i] || !Y[i] || ldx[i] < N[i] || ldy[i] < N[i] || X[i] == Y[i])
      return berr(b, CF_EINVAL, "filter_batch: bad block " + std::to_string(i));
    if (!std::isfinite(a[i]) || !std::isfinite(bu[i]) || !(bu[i] > a[i]))
      return berr(b, CF_EINVAL, "filter_batch: need finite a < b for entry " + std::to_string(i));
  }
  BHIPCHK(b, hipSetDevice(b->device));
  if (prec == CF_FP64 || m == 0) {
    // FP64 (or degree 0): the single-problem path entry by entry
    for (int i = 0; i < b->count; ++i) {
      cf_ctx *c = b->uniq[b->which[i]];
      cf_status st = chebfilter_filter(c, X[i], ldx[i], Y[i], ldy[i], N[i], m, a[i], bu[i], CF_FP64);
      if (st != CF_OK) return berr(b, st, "entry " + std::to_string(i) + ": " + c->err);
    }
    return CF_OK;
  }
  const bool bf16 = prec == CF_BF16;
  STCHK(batch_prepare_lowp(b, bf16, m));
  // per-call descriptor fields, staged in pinned memory (wait for the previous copy)
  if (b->copy_pending) BHIPCHK(b, hipEventSynchronize(b->ev_copy));
  for (int i = 0; i < b->count; ++i) {
    BatchProb P = b->h_bp[i];
    P.X = X[i]; P.ldx = ldx[i]; P.Y = Y[i]; P.ldy = ldy[i]; P.N = (int)N[i];
    P.e = 2.0 / (bu[i] - a[i]);
    P.cc = (a[i] + bu[i]) / (bu[i] - a[i]);
    b->stage[i] = P;
  }
  BHIPCHK(b, hipEventRecord(b->ev_in, b->caller));
  BHIPCHK(b, hipStreamWaitEvent(b->bs, b->ev_in, 0));
  BHIPCHK(b, hipMemcpyAsync(b->d_bp, b->stage, (size_t)b->count * sizeof(BatchProb),
                            hipMemcpyHostToDevice, b->bs));
  BHIPCHK(b, hipEventRecord(b->ev_copy, b->bs));
  b->copy_pending = true;
  if (use_graph) {
    const int nsb_key = (4 * b->nsb[0] + b->nsb[1]) | (b->bmap << 8);
    if (!b->gexec || b->g_m != m || b->g_prec != prec || b->g_nsb != nsb_key) {
      if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
      hipGraph_t g = nullptr;
      BHIPCHK(b, hipStreamBeginCapture(b->bs, hipStreamCaptureModeThreadLocal));
      cf_status st = batch_enqueue_filter(b, m, bf16);
      hipError_t ec = hipStreamEndCapture(b->bs, &g);
      if (st != CF_OK) { if (g) (void)hipGraphDestroy(g); return st; }
      if (ec != hipSuccess) return berr(b, CF_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
      ec = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ec != hipSuccess) {
        b->gexec = nullptr;
        return berr(b, CF_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
      }
      b->g_m = m;
      b->g_prec = prec;
      b->g_nsb = nsb_key;
    }
    BHIPCHK(b, hipGraphLaunch(b->gexec, b->bs));
  } else {
    STCHK(batch_enqueue_filter(b, m, bf16));
  }
  BHIPCHK(b, hipEventRecord(b->ev_out, b->bs));
  BHIPCHK(b, hipStreamWaitEvent(b->caller, b->ev_out, 0));
  return CF_OK;
}

cf_status chebfilter_set_cell_tile(cf_ctx *c, int32_t prec, int32_t nsb) {
  if (!c) return CF_EINVAL;
  if (prec != CF_FP32 && prec != CF_BF16) return set_err(c, CF_EINVAL, "set_cell_tile: prec must be CF_FP32 or CF_BF16");
  if (nsb != 1 && nsb != 2) return set_err(c, CF_EINVAL, "set_cell_tile: nsb must be 1 or 2");
  c->lp_nsb[prec == CF_BF16 ? 1 : 0] = nsb;
  return CF_OK;
}

// Time `reps` filters after one warm-up for each candidate, keep the fastest
// (HIP events on the context's stream): first the reduced cell product's
// column blocks per tile, then, bucket by bucket (cells with 1, 2, 3, >= 4
// blocks of 16 enrichment functions), the split of the FP32 coupling
// partials' waves between row blocks and k parts (greedy: each bucket with
// the others fixed).
extern "C++" {
template <typename Run>
static cf_status tune_loop(hipStream_t s, int reps, Run run, float *ms_out) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return CF_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return CF_EDEVICE; }
  cf_status st = run();
  if (st == CF_OK) {
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == CF_OK; ++r) st = run();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Greedy bucket search of the coupling map: `map` is updated in place.
template <typename Run>
static cf_status tune_bmap(hipStream_t s, int reps, int *map, Run run) {
  float best = 0.f;
  cf_status st = tune_loop(s, reps, run, &best);
  for (int q = 0; q < 4 && st == CF_OK; ++q) {
    const int keep = *map;
    int best_map = keep;
    for (int code = 0; code < 3 && st == CF_OK; ++code) {
      const int cand = (keep & ~(3 << (2 * q))) | (code << (2 * q));
      if (cand == keep) continue;
      *map = cand;
      float ms = 0.f;
      st = tune_loop(s, reps, run, &ms);
      if (st == CF_OK && ms < best) { best = ms; best_map = cand; }
    }
    *map = best_map;
  }
  return st;
}
}  // extern "C++"

cf_status chebfilter_autotune(cf_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                              int64_t N, int32_t m, double a, double b, int32_t prec, int32_t reps,
                              int32_t *choice) {
  if (!c) return CF_EINVAL;
  if (prec != CF_FP32 && prec != CF_BF16) return set_err(c, CF_EINVAL, "autotune: prec must be CF_FP32 or CF_BF16");
  if (reps < 1 || m < 1) return set_err(c, CF_EINVAL, "autotune: need reps >= 1 and m >= 1");
  HIPCHK(c, hipSetDevice(c->device));
  const int slot = prec == CF_BF16 ? 1 : 0;
  auto run = [&]() { return chebfilter_filter(c, X, ldx, Y, ldy, N, m, a, b, prec); };
  float best = 0.f;
  int best_nsb = c->lp_nsb[slot];
  cf_status st = CF_OK;
  for (int nsb = 1; nsb <= 2 && st == CF_OK; ++nsb) {
    c->lp_nsb[slot] = nsb;
    float ms = 0.f;
    st = tune_loop(c->stream, reps, run, &ms);
    if (st == CF_OK && (nsb == 1 || ms < best)) { best = ms; best_nsb = nsb; }
  }
  c->lp_nsb[slot] = best_nsb;
  if (st == CF_OK && c->n_e > 0) st = tune_bmap(c->stream, reps, &c->lp_bmap, run);
  if (st != CF_OK) return st == CF_EDEVICE ? set_err(c, st, "autotune: event") : st;
  if (choice) *choice = best_nsb;
  return CF_OK;
}

cf_status chebfilter_tuning(cf_ctx *c, int32_t set_map, int32_t *nsb_fp32, int32_t *nsb_bf16,
                            int32_t *coupling_map) {
  if (!c) return CF_EINVAL;
  if (set_map >= 0) {
    if (set_map > 255 || ((set_map & 0x55) & (set_map >> 1) & 0x55))
      return set_err(c, CF_EINVAL, "tuning: coupling map codes must be 0, 1 or 2");
    c->lp_bmap = set_map;
  }
  if (nsb_fp32) *nsb_fp32 = c->lp_nsb[0];
  if (nsb_bf16) *nsb_bf16 = c->lp_nsb[1];
  if (coupling_map) *coupling_map = c->lp_bmap;
  return CF_OK;
}

cf_status chebfilter_batch_autotune(cf_batch *b, const double *const *X, const int64_t *ldx,
                                    double *const *Y, const int64_t *ldy, const int64_t *N,
                                    int32_t m, const double *a, const double *bu, int32_t prec,
                                    int32_t reps, int32_t *choice) {
  if (!b) return CF_EINVAL;
  if (prec != CF_FP32 && prec != CF_BF16) return berr(b, CF_EINVAL, "batch_autotune: prec must be CF_FP32 or CF_BF16");
  if (reps < 1 || m < 1) return berr(b, CF_EINVAL, "batch_autotune: need reps >= 1 and m >= 1");
  BHIPCHK(b, hipSetDevice(b->device));
  const int slot = prec == CF_BF16 ? 1 : 0;
  auto run = [&]() { return chebfilter_filter_batch(b, X, ldx, Y, ldy, N, m, a, bu, prec, 1); };
  float best = 0.f;
  int best_nsb = b->nsb[slot];
  cf_status st = CF_OK;
  for (int nsb = 1; nsb <= 2 && st == CF_OK; ++nsb) {
    b->nsb[slot] = nsb;
    float ms = 0.f;
    st = tune_loop(b->caller, reps, run, &ms);
    if (st == CF_OK && (nsb == 1 || ms < best)) { best = ms; best_nsb = nsb; }
  }
  b->nsb[slot] = best_nsb;
  if (st == CF_OK && b->neitems > 0) st = tune_bmap(b->caller, reps, &b->bmap, run);
  if (st != CF_OK) return st == CF_EDEVICE ? berr(b, st, "batch_autotune: event") : st;
  if (choice) *choice = best_nsb;
  return CF_OK;
}

cf_status chebfilter_batch_tuning(cf_batch *b, int32_t set_map, int32_t *nsb_fp32,
                                  int32_t *nsb_bf16, int32_t *coupling_map) {
  if (!b) return CF_EINVAL;
  if (set_map >= 0) {
    if (set_map > 255 || ((set_map & 0x55) & (set_map >> 1) & 0x55))
      return berr(b, CF_EINVAL, "batch_tuning: coupling map codes must be 0, 1 or 2");
    b->bmap = set_map;
  }
  if (nsb_fp32) *nsb_fp32 = b->nsb[0];
  if (nsb_bf16) *nsb_bf16 = b->nsb[1];
  if (coupling_map) *coupling_map = b->bmap;
  return CF_OK;
}

static cf_status batch_rr_alloc(cf_batch *b) {
  if (b->d_rst) return CF_OK;
  const size_t cnt = (size_t)b->count, mc = (size_t)b->max_cols;
  STCHK(balloc(b, &b->d_rst, 8 * cnt));
  STCHK(balloc(b, &b->d_rinfo, cnt));
  STCHK(balloc(b, &b->d_rslot, cnt));
  STCHK(balloc(b, &b->d_rH, cnt * mc * mc));
  STCHK(balloc(b, &b->d_rM, cnt * mc * mc));
  STCHK(balloc(b, &b->d_rth, cnt * mc));
  STCHK(balloc(b, &b->d_rE, cnt * mc));
  STCHK(balloc(b, &b->d_lz, 2 * cnt));
  b->h_rslot.assign(cnt, -1);
  b->h_rst.assign(8 * cnt, 0);
  b->h_rth.assign(cnt * mc, 0.0);
  b->h_lz.assign(2 * cnt, 0.0);
  return CF_OK;
}

// Every entry is projected with no host wait: two unshifted Cholesky-QR
// passes whose failure flags land in the entry's status words (the result
// reaches the block through a predicated copy, so a failed pass leaves it as
// it was), the projected pencil into the entry's slot, then one batched
// generalized eigensolve per block width and the rotation, again through a
// predicated copy.  One synchronisation reads every status; an entry whose
// orthonormalisation or eigensolve failed is redone by the single-problem
// projection (shifted Cholesky-QR, its own error reporting) on its block,
// which still spans the filtered subspace.  Status words per entry: [0], [1]
// the two Cholesky passes, [2] the eigensolver's info, [3] a non-finite
// pencil, [4] a non-finite rotated block, [5], [6] a bad Gram diagonal in
// the two passes.
cf_status chebfilter_rayleigh_ritz_batch(cf_batch *b, double *const *Y, const int64_t *ldy,
                                         const int64_t *N, double *const *theta_host) {
  if (!b) return CF_EINVAL;
  if (!Y || !ldy || !N || !theta_host) return berr(b, CF_EINVAL, "rayleigh_ritz_batch: null argument array");
  for (int i = 0; i < b->count; ++i) {
    cf_ctx *c = b->uniq[b->which[i]];
    cf_status st = check_block(c, Y[i], ldy[i], N[i], "rayleigh_ritz_batch Y");
    if (st == CF_OK && N[i] > 0 && !theta_host[i])
      st = set_err(c, CF_EINVAL, "rayleigh_ritz_batch: null theta");
    if (st != CF_OK) return berr(b, st, "entry " + std::to_string(i) + ": " + c->err);
  }
  BHIPCHK(b, hipSetDevice(b->device));
  STCHK(batch_rr_alloc(b));
  const int cnt = b->count;
  const int64_t mc = b->max_cols, mc2 = mc * mc;
  // slots: entries with columns, ordered by width (stable), so that each
  // width's pencils are contiguous for the strided batched eigensolver
  std::vector<int> order;
  for (int i = 0; i < cnt; ++i)
    if (N[i] > 0) order.push_back(i);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return N[x] < N[y]; });
  std::fill(b->h_rslot.begin(), b->h_rslot.end(), -1);
  for (size_t k = 0; k < order.size(); ++k) b->h_rslot[order[k]] = (int)k;
  if (order.empty()) return CF_OK;
  cf_ctx *c0 = b->uniq[0];
  hipStream_t s = c0->stream;
  BHIPCHK(b, hipMemsetAsync(b->d_rst, 0, 8 * (size_t)cnt * sizeof(int), s));
  BHIPCHK(b, hipMemcpyAsync(b->d_rslot, b->h_rslot.data(), (size_t)cnt * sizeof(int),
                            hipMemcpyHostToDevice, s));
  auto fail = [&](int i, cf_ctx *c, cf_status st) {
    return berr(b, st, "entry " + std::to_string(i) + ": " + c->err);
  };
  // orthonormalisation and projected pencils
  for (int i : order) {
    cf_ctx *c = b->uniq[b->which[i]];
    const int n = (int)N[i];
    const int64_t ld = c->ldw;
    int *st = b->d_rst + 8 * i;
    double *Hh = b->d_rH + b->h_rslot[i] * mc2, *Mh = b->d_rM + b->h_rslot[i] * mc2;
    cf_status r = CF_OK;
    // the steps of core_cholqr_pass (scaling kernel, library Cholesky and
    // rotation), so that both paths compute the same basis; pass 0 writes the
    // scratch block T, pass 1 writes U and is copied into Y only if both
    // passes succeeded
    for (int pass = 0; pass < 2 && r == CF_OK; ++pass) {
      const double *In = pass == 0 ? Y[i] : c->T;
      const int64_t ldi = pass == 0 ? ldy[i] : ld;
      r = core_gram(c, In, ldi, In, ldi, c->n, n, c->G, GRAM_UPPER);
      if (r != CF_OK) break;
      if (launch_chol_scale(s, c->G, n, 0.0, c->sv, st + 5 + pass) != hipSuccess ||
          rocsolver_dpotrf(c->rb, rocblas_fill_upper, n, c->G, n, (rocblas_int *)(st + pass)) !=
              rocblas_status_success ||
          launch_tri_inv_T(s, c->G, c->sv, n, c->Wm) != hipSuccess)
        r = set_err(c, CF_EDEVICE, "rayleigh_ritz_batch: launch failed");
      if (r == CF_OK) r = core_rotate(c, In, ldi, c->Wm, n, pass == 0 ? c->T : c->U, ld);
    }
    if (r == CF_OK && launch_copy_skip(s, c->n, n, c->U, ld, Y[i], ldy[i], st) != hipSuccess)
      r = set_err(c, CF_EDEVICE, "rayleigh_ritz_batch: launch failed");
    if (r == CF_OK) r = core_apply_H(c, Y[i], ldy[i], c->T, ld, n);
    if (r == CF_OK) r = core_gram(c, Y[i], ldy[i], c->T, ld, c->n, n, Hh, GRAM_SYM);
    if (r == CF_OK) r = core_apply_M(c, Y[i], ldy[i], c->T, ld, n);
    if (r == CF_OK) r = core_gram(c, Y[i], ldy[i], c->T, ld, c->n, n, Mh, GRAM_SYM);
    if (r == CF_OK && launch_rr_guard(s, Hh, Mh, n, st) != hipSuccess)
      r = set_err(c, CF_EDEVICE, "rayleigh_ritz_batch: guard launch failed");
    if (r != CF_OK) return fail(i, c, r);
  }
  // one generalized eigensolve per width over its contiguous slots
  for (size_t k0 = 0; k0 < order.size();) {
    size_t k1 = k0;
    while (k1 < order.size() && N[order[k1]] == N[order[k0]]) ++k1;
    const int n = (int)N[order[k0]];
    if (rocsolver_dsygvd_strided_batched(c0->rb, rocblas_eform_ax, rocblas_evect_original,
                                         rocblas_fill_upper, n, b->d_rH + k0 * mc2, n, mc2,
                                         b->d_rM + k0 * mc2, n, mc2, b->d_rth + k0 * mc, mc,
                                         b->d_rE + k0 * mc, mc, b->d_rinfo + k0,
                                         (rocblas_int)(k1 - k0)) != rocblas_status_success)
      return berr(b, CF_EDEVICE, "rayleigh_ritz_batch: rocsolver_dsygvd_strided_batched failed");
    k0 = k1;
  }
  BHIPCHK(b, launch_rr_info(s, b->d_rinfo, b->d_rslot, cnt, b->d_rst));
  // predicated rotation Y <- Q V through the context's scratch block
  for (int i : order) {
    cf_ctx *c = b->uniq[b->which[i]];
    const int n = (int)N[i];
    const int64_t ld = c->ldw;
    int *st = b->d_rst + 8 * i;
    BHIPCHK(b, launch_transpose(s, n, b->d_rH + b->h_rslot[i] * mc2, n, c->Wm));
    {
      cf_status r = core_rotate(c, Y[i], ldy[i], c->Wm, n, c->T, ld);
      if (r != CF_OK) return fail(i, c, r);
    }
    BHIPCHK(b, launch_copy_skip(s, c->n, n, c->T, ld, Y[i], ldy[i], st));
    if (c->check_finite) BHIPCHK(b, launch_check_finite(s, Y[i], ldy[i], c->n, n, st + 4));
  }
  BHIPCHK(b, hipMemcpyAsync(b->h_rst.data(), b->d_rst, 8 * (size_t)cnt * sizeof(int),
                            hipMemcpyDeviceToHost, s));
  BHIPCHK(b, hipMemcpyAsync(b->h_rth.data(), b->d_rth, (size_t)cnt * mc * sizeof(double),
                            hipMemcpyDeviceToHost, s));
  BHIPCHK(b, hipStreamSynchronize(s));
  for (int i = 0; i < cnt; ++i) {
    if (N[i] == 0) continue;
    cf_ctx *c = b->uniq[b->which[i]];
    const int *st = b->h_rst.data() + 8 * i;
    if (st[3]) return fail(i, c, set_err(c, CF_ENUMERIC, "rayleigh_ritz_batch: non-finite projected pencil"));
    if (st[0] | st[1] | st[2] | st[5] | st[6]) {
      cf_status r = chebfilter_rayleigh_ritz(c, Y[i], ldy[i], N[i], theta_host[i]);
      if (r != CF_OK) return fail(i, c, r);
      continue;
    }
    if (st[4]) return fail(i, c, set_err(c, CF_ENUMERIC, "rayleigh_ritz_batch: non-finite values in the output"));
    std::memcpy(theta_host[i], b->h_rth.data() + b->h_rslot[i] * mc, (size_t)N[i] * sizeof(double));
  }
  return CF_OK;
}

static constexpr int LZ_CHUNKS = 128;   // row chunks of the column dot products

static cf_status batch_lz_alloc(cf_batch *b) {
  if (b->d_lzblk) return CF_OK;
  for (size_t u = 0; u < b->uniq.size(); ++u) {
    std::vector<int> g;
    for (int i = 0; i < b->count; ++i) {
      if (b->which[i] != (int)u) continue;
      g.push_back(i);
      if ((int64_t)g.size() == b->max_cols) { b->lz_groups.push_back(g); g.clear(); }
    }
    if (!g.empty()) b->lz_groups.push_back(g);
    b->lz_n = std::max<int64_t>(b->lz_n, b->uniq[u]->n);
  }
  for (auto &g : b->lz_groups) b->lz_k = std::max<int>(b->lz_k, (int)g.size());
  STCHK(balloc(b, &b->d_lzblk, 4 * (size_t)b->lz_n * b->lz_k));
  STCHK(balloc(b, &b->d_lzc, (2 * 64 + 8) * (size_t)b->lz_k));
  STCHK(balloc(b, &b->d_lzp, (size_t)LZ_CHUNKS * b->lz_k));
  return CF_OK;
}

// k Lanczos steps of every entry.  The runs of the entries that share a
// problem are the columns of one n x r block, so each step applies the
// operator once per problem (Sec. V's estimate, run for r start vectors at
// once; the runs stay independent: column-wise dot products and updates);
// all groups are enqueued back to back and one wait reads every bound.
cf_status chebfilter_lanczos_bounds_batch(cf_batch *b, const double *const *v0, int32_t k,
                                          double *lmin_est, double *b_upper) {
  if (!b) return CF_EINVAL;
  if (!v0 || !lmin_est || !b_upper) return berr(b, CF_EINVAL, "lanczos_bounds_batch: null argument array");
  if (k < 1 || k > 64) return berr(b, CF_EINVAL, "lanczos_bounds_batch: k must be 1..64");
  for (int i = 0; i < b->count; ++i)
    if (!v0[i]) return berr(b, CF_EINVAL, "entry " + std::to_string(i) + ": null v0");
  BHIPCHK(b, hipSetDevice(b->device));
  STCHK(batch_rr_alloc(b));
  STCHK(batch_lz_alloc(b));
  hipStream_t s = b->uniq[0]->stream;
  std::vector<int> slot_entry;
  for (const auto &g : b->lz_groups) {
    cf_ctx *c = b->uniq[b->which[g[0]]];
    const int r = (int)g.size();
    const int64_t n = c->n;
    double *vprev = b->d_lzblk, *v = vprev + n * r, *w = v + n * r, *mv = w + n * r;
    double *coef = b->d_lzc;
    auto fail = [&](cf_status st) {
      return berr(b, st, "entry " + std::to_string(g[0]) + ": " + c->err);
    };
    cf_status st = CF_OK;
    for (int t = 0; t < r; ++t) BHIPCHK(b, launch_copy(s, n, 1, v0[g[t]], 1, w + t, r));
    BHIPCHK(b, hipMemsetAsync(coef, 0, (2 * 64 + 8) * (size_t)r * sizeof(double), s));
    if ((st = core_apply_M(c, w, r, mv, r, r)) != CF_OK) return fail(st);
    BHIPCHK(b, launch_coldot(s, n, r, w, r, mv, r, b->d_lzp, LZ_CHUNKS, coef));
    BHIPCHK(b, launch_lanczos_update_blk(s, n, r, 0, w, nullptr, nullptr, coef, v, 0));
    for (int j = 0; j < k; ++j) {
      if ((st = core_htilde_step(c, v, r, r, 1.0, nullptr, 0, 0.0, nullptr, 0, 0.0, w, r)) != CF_OK)
        return fail(st);
      if (j > 0) BHIPCHK(b, launch_lanczos_update_blk(s, n, r, j, w, v, vprev, coef, nullptr, 1));
      if ((st = core_apply_M(c, v, r, mv, r, r)) != CF_OK) return fail(st);
      BHIPCHK(b, launch_coldot(s, n, r, w, r, mv, r, b->d_lzp, LZ_CHUNKS, coef + (1 + 2 * j) * r));
      BHIPCHK(b, launch_lanczos_update_blk(s, n, r, j, w, v, vprev, coef, nullptr, 2));
      if ((st = core_apply_M(c, w, r, mv, r, r)) != CF_OK) return fail(st);
      BHIPCHK(b, launch_coldot(s, n, r, w, r, mv, r, b->d_lzp, LZ_CHUNKS, coef + (2 + 2 * j) * r));
      if (j + 1 < k) {
        BHIPCHK(b, launch_lanczos_update_blk(s, n, r, j, w, v, vprev, coef, vprev, 3));
        std::swap(vprev, v);
      }
    }
    BHIPCHK(b, launch_tridiag_bounds_blk(s, coef, r, k, b->d_lz + 2 * slot_entry.size()));
    slot_entry.insert(slot_entry.end(), g.begin(), g.end());
  }
  BHIPCHK(b, hipMemcpyAsync(b->h_lz.data(), b->d_lz, 2 * (size_t)b->count * sizeof(double),
                            hipMemcpyDeviceToHost, s));
  BHIPCHK(b, hipStreamSynchronize(s));
  for (size_t q = 0; q < slot_entry.size(); ++q) {
    const int i = slot_entry[q];
    lmin_est[i] = b->h_lz[2 * q];
    b_upper[i] = b->h_lz[2 * q + 1];
  }
  for (int i = 0; i < b->count; ++i)
    if (!std::isfinite(lmin_est[i]) || !std::isfinite(b_upper[i]))
      return berr(b, CF_ENUMERIC, "entry " + std::to_string(i) + ": non-finite Lanczos bound (breakdown?)");
  return CF_OK;
}

// ---------------------------------------------------------------------------
// operator updates, residuals, learned bounds
// ---------------------------------------------------------------------------
cf_status chebfilter_update_H_cc(cf_ctx *c, const double *H_cc) {
  if (!c) return CF_EINVAL;
  if (!H_cc) return set_err(c, CF_EINVAL, "update_H_cc: null H_cc");
  HIPCHK(c, hipSetDevice(c->device));
  return upload_cells(c, H_cc, "update_H_cc");
}

cf_status chebfilter_assembly_tables(cf_ctx *c, int32_t nq, const double *B, const double *w,
                                     const double *K) {
  if (!c) return CF_EINVAL;
  if (nq < 1 || nq > 4096) return set_err(c, CF_EINVAL, "assembly_tables: nq must be 1..4096");
  if (!B || !w || !K) return set_err(c, CF_EINVAL, "assembly_tables: null table");
  const int npc = c->npc;
  const int nq4 = (nq + 3) & ~3;
  std::vector<double> hB((size_t)nq4 * NPAD, 0.0), hK((size_t)NPAD * NPAD, 0.0);
  double kmax = 0.0;
  for (int64_t q = 0; q < (int64_t)nq * npc; ++q)
    if (!std::isfinite(B[q])) return set_err(c, CF_EINVAL, "assembly_tables: non-finite B");
  for (int q = 0; q < nq; ++q) {
    if (!std::isfinite(w[q])) return set_err(c, CF_EINVAL, "assembly_tables: non-finite w");
    for (int a = 0; a < npc; ++a) hB[(size_t)q * NPAD + a] = B[(size_t)q * npc + a];
  }
  for (int64_t q = 0; q < (int64_t)npc * npc; ++q) {
    if (!std::isfinite(K[q])) return set_err(c, CF_EINVAL, "assembly_tables: non-finite K");
    kmax = std::max(kmax, std::fabs(K[q]));
  }
  for (int a = 0; a < npc; ++a)
    for (int b = 0; b < npc; ++b) {
      const double x = K[a * npc + b], y = K[b * npc + a];
      if (std::fabs(x - y) > 1e-10 * kmax) return set_err(c, CF_EINVAL, "assembly_tables: K not symmetric");
      hK[(size_t)a * NPAD + b] = 0.5 * (x + y);
    }
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->asm_nq < nq4) {
    if (c->asm_B) { (void)hipFree(c->asm_B); c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void *)c->asm_B)); c->asm_B = nullptr; }
    if (c->asm_w) { (void)hipFree(c->asm_w); c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void *)c->asm_w)); c->asm_w = nullptr; }
  }
  if (!c->asm_B) {
    STCHK(dalloc(c, &c->asm_B, hB.size()));
    STCHK(dalloc(c, &c->asm_w, (size_t)nq4));
  }
  if (!c->asm_K) STCHK(dalloc(c, &c->asm_K, hK.size()));
  HIPCHK(c, hipMemcpy(c->asm_B, hB.data(), hB.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->asm_w, w, (size_t)nq * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->asm_K, hK.data(), hK.size() * sizeof(double), hipMemcpyHostToDevice));
  c->asm_nq = nq;
  return CF_OK;
}

cf_status chebfilter_assemble_cells(cf_ctx *c, const int32_t *cells, int64_t ncells, const double *V,
                                    int64_t ldv) {
  if (!c) return CF_EINVAL;
  if (!c->asm_B) return set_err(c, CF_EINVAL, "assemble_cells: no reference tables (chebfilter_assembly_tables)");
  if (ncells < 0 || ncells > c->E) return set_err(c, CF_EINVAL, "assemble_cells: bad cell count");
  if (ncells == 0) return CF_OK;
  if (!cells || !V) return set_err(c, CF_EINVAL, "assemble_cells: null argument");
  if (ldv < c->asm_nq) return set_err(c, CF_EINVAL, "assemble_cells: ldv < nq");
  std::vector<uint8_t> seen(c->E, 0);
  for (int64_t i = 0; i < ncells; ++i) {
    const int32_t e = cells[i];
    if (e < 0 || e >= c->E) return set_err(c, CF_EINVAL, "assemble_cells: cell index out of range");
    if (c->cell_enriched[e])
      return set_err(c, CF_EINVAL, "assemble_cells: cell " + std::to_string(e) +
                                       " carries enrichment functions (its blocks use the adaptive rule)");
    if (seen[e]) return set_err(c, CF_EINVAL, "assemble_cells: cell listed twice");
    seen[e] = 1;
  }
  HIPCHK(c, hipSetDevice(c->device));
  if ((int64_t)c->asm_list.size() != ncells ||
      !std::equal(c->asm_list.begin(), c->asm_list.end(), cells)) {
    // a new cell list: wait for work that may still read the old one
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (ncells > c->asm_cap) {
      if (c->asm_cells) {
        (void)hipFree(c->asm_cells);
        c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void *)c->asm_cells));
        c->asm_cells = nullptr;
      }
      STCHK(dalloc(c, &c->asm_cells, (size_t)ncells));
      c->asm_cap = ncells;
    }
    HIPCHK(c, hipMemcpy(c->asm_cells, cells, (size_t)ncells * sizeof(int32_t), hipMemcpyHostToDevice));
    c->asm_list.assign(cells, cells + ncells);
  }
  {
    Scope sc(c, "assemble", 2.0 * 36 * 256 * (double)((c->asm_nq + 3) & ~3) * ncells);
    HIPCHK(c, launch_assemble_cells(c->stream, c->asm_B, c->asm_w, c->asm_K, c->asm_cells,
                                    (int)ncells, V, ldv, c->asm_nq, c->Hp));
  }
  const int64_t hsz = c->E * NPAD * NPAD;
  if (c->Hp32) HIPCHK(c, launch_to_f32(c->stream, hsz, c->Hp, c->Hp32));
  if (c->Hp16) HIPCHK(c, launch_to_bf16(c->stream, hsz, c->Hp, c->Hp16));
  return CF_OK;
}

// ---------------------------------------------------------------------------
// Element blocks of the cells with their own adaptive rule (Sec. IV.C)
// ---------------------------------------------------------------------------
extern "C++" {
template <class T>
static void dfree(cf_ctx *c, T *&p) {
  if (!p) return;
  (void)hipFree((void *)p);
  auto it = std::find(c->allocs.begin(), c->allocs.end(), (void *)p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  p = nullptr;
}

template <class T>
static cf_status dupload(cf_ctx *c, T *&p, const T *host, size_t count) {
  dfree(c, p);
  STCHK(dalloc(c, &p, std::max<size_t>(count, 1)));
  if (count) HIPCHK(c, hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice));
  return CF_OK;
}
}  // extern "C++"

// partial H^ee blocks of one batch of enriched cells stay below this
static constexpr int64_t EA_PEE_BYTES = 512ll << 20;

cf_status chebfilter_enriched_tables(cf_ctx *c, const cf_adaptive_grid *g) {
  if (!c) return CF_EINVAL;
  if (!g) return set_err(c, CF_EINVAL, "enriched_tables: null grid");
  if (!c->asm_K) return set_err(c, CF_EINVAL, "enriched_tables: no kinetic block (chebfilter_assembly_tables)");
  const int64_t ncl = g->ncells;
  if (ncl < 1 || ncl > c->E) return set_err(c, CF_EINVAL, "enriched_tables: bad cell count");
  if (!g->cells || !g->cell_lo || !g->nodes || !g->gauss_x || !g->gauss_w || !g->box_ptr ||
      !g->box_lo || !g->box_size)
    return set_err(c, CF_EINVAL, "enriched_tables: null array");
  const int np1 = g->n_nodes, ng = g->ng;
  if (np1 < 2 || np1 > EA_MAXNP || np1 * np1 * np1 != c->npc)
    return set_err(c, CF_EINVAL, "enriched_tables: n_nodes^3 must equal the cell's node count (n_nodes <= 8)");
  if (ng < 1 || ng > 8) return set_err(c, CF_EINVAL, "enriched_tables: ng must be 1..8");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return set_err(c, CF_EINVAL, "enriched_tables: bad h");
  for (int i = 0; i < np1; ++i)
    if (!std::isfinite(g->nodes[i]) || (i && !(g->nodes[i] > g->nodes[i - 1])))
      return set_err(c, CF_EINVAL, "enriched_tables: nodes must be finite and increasing");
  double wsum = 0.0;
  for (int i = 0; i < ng; ++i) {
    if (!(g->gauss_x[i] > 0.0 && g->gauss_x[i] < 1.0) || !std::isfinite(g->gauss_w[i]))
      return set_err(c, CF_EINVAL, "enriched_tables: Gauss points must lie in (0, 1)");
    wsum += g->gauss_w[i];
  }
  if (std::fabs(wsum - 1.0) > 1e-12) return set_err(c, CF_EINVAL, "enriched_tables: Gauss weights must sum to 1");
  // cells: distinct, in range, every cell with enrichment functions listed
  std::vector<uint8_t> seen(c->E, 0);
  for (int64_t i = 0; i < ncl; ++i) {
    const int32_t e = g->cells[i];
    if (e < 0 || e >= c->E) return set_err(c, CF_EINVAL, "enriched_tables: cell index out of range");
    if (seen[e]) return set_err(c, CF_EINVAL, "enriched_tables: cell listed twice");
    seen[e] = 1;
  }
  if (c->n_e > 0)
    for (int64_t e = 0; e < c->E; ++e)
      if (c->cell_enriched[e] && !seen[e])
        return set_err(c, CF_EINVAL, "enriched_tables: cell " + std::to_string(e) +
                                         " carries enrichment functions but is not listed");
  // boxes: at least one per cell, positive sides, inside the cell
  if (g->box_ptr[0] != 0) return set_err(c, CF_EINVAL, "enriched_tables: box_ptr[0] must be 0");
  for (int64_t i = 0; i < ncl; ++i)
    if (g->box_ptr[i + 1] <= g->box_ptr[i]) return set_err(c, CF_EINVAL, "enriched_tables: a cell without boxes");
  const int64_t nbox = g->box_ptr[ncl];
  const int64_t ng3 = (int64_t)ng * ng * ng;
  if (nbox > ((int64_t)1 << 40) / ng3) return set_err(c, CF_EINVAL, "enriched_tables: too many points");
  for (int64_t i = 0; i < ncl; ++i) {
    const double *lo = g->cell_lo + 3 * i;
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(lo[d])) return set_err(c, CF_EINVAL, "enriched_tables: non-finite cell corner");
    const double tol = 1e-9 * g->h;
    for (int64_t b = g->box_ptr[i]; b < g->box_ptr[i + 1]; ++b) {
      const double s = g->box_size[b];
      if (!(s > 0.0) || !std::isfinite(s)) return set_err(c, CF_EINVAL, "enriched_tables: bad box side");
      for (int d = 0; d < 3; ++d) {
        const double bl = g->box_lo[3 * b + d];
        if (!std::isfinite(bl) || bl < lo[d] - tol || bl + s > lo[d] + g->h + tol)
          return set_err(c, CF_EINVAL, "enriched_tables: box " + std::to_string(b) + " outside its cell");
      }
    }
  }
  // enrichment description
  const int nsh = g->n_shells;
  int npa = 0, nterm = 0;
  if (c->n_e > 0) {
    if (g->n_atoms < 1 || !g->centers || nsh < 1 || !g->shell_l || !g->shell_term_ptr ||
        !g->term_c || !g->term_k || !g->term_zeta)
      return set_err(c, CF_EINVAL, "enriched_tables: enrichment description missing");
    if (!(g->r0 > 0.0) || !(g->t > 0.0) || !std::isfinite(g->r0) || !std::isfinite(g->t))
      return set_err(c, CF_EINVAL, "enriched_tables: bad cutoff (r0, t)");
    if (g->shell_term_ptr[0] != 0) return set_err(c, CF_EINVAL, "enriched_tables: shell_term_ptr[0] must be 0");
    for (int s = 0; s < nsh; ++s) {
      const int l = g->shell_l[s];
      if (l != 0 && l != 1) return set_err(c, CF_EINVAL, "enriched_tables: shells must have l = 0 or 1");
      npa += 2 * l + 1;
      if (g->shell_term_ptr[s + 1] <= g->shell_term_ptr[s])
        return set_err(c, CF_EINVAL, "enriched_tables: a shell without radial terms");
      for (int k = g->shell_term_ptr[s]; k < g->shell_term_ptr[s + 1]; ++k)
        if (!std::isfinite(g->term_c[k]) || !(g->term_zeta[k] >= 0.0) || g->term_k[k] < l ||
            g->term_k[k] > 16)
          return set_err(c, CF_EINVAL, "enriched_tables: bad radial term (k >= l, k <= 16, zeta >= 0)");
    }
    nterm = g->shell_term_ptr[nsh];
    if (npa > 16) return set_err(c, CF_EINVAL, "enriched_tables: more than 16 functions per atom");
    if ((int64_t)g->n_atoms * npa != c->n_e)
      return set_err(c, CF_EINVAL, "enriched_tables: n_atoms * functions per atom != n_e");
    for (int64_t q = 0; q < 3 * (int64_t)g->n_atoms; ++q)
      if (!std::isfinite(g->centers[q])) return set_err(c, CF_EINVAL, "enriched_tables: non-finite centre");
  }
  if (ea_tab_size(np1, ng, nsh, nterm) > EA_TAB_MAX)
    return set_err(c, CF_EINVAL, "enriched_tables: too many shells or radial terms");

  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // the context's enrichment lists (host copies)
  std::vector<int64_t> ep;
  std::vector<int32_t> eidx;
  if (c->n_e > 0) {
    ep.resize(c->E + 1);
    HIPCHK(c, hipMemcpy(ep.data(), c->eptr, (c->E + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    eidx.resize(std::max<int64_t>(ep[c->E], 1));
    if (ep[c->E]) HIPCHK(c, hipMemcpy(eidx.data(), c->eidx, ep[c->E] * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  // per listed cell: its atoms (complete groups of npa functions, ascending)
  std::vector<std::vector<int32_t>> atoms(ncl);
  for (int64_t i = 0; i < ncl && c->n_e > 0; ++i) {
    const int32_t e = g->cells[i];
    const int64_t na = ep[e + 1] - ep[e];
    if (na == 0) continue;
    if (na % npa || na > EA_MAXNAP)
      return set_err(c, CF_EINVAL, "enriched_tables: cell " + std::to_string(e) +
                                       ": its functions are not whole atoms (or more than 256)");
    for (int64_t u = 0; u < na / npa; ++u) {
      const int32_t f0 = eidx[ep[e] + u * npa];
      if (f0 % npa) return set_err(c, CF_EINVAL, "enriched_tables: function groups not atom-aligned");
      for (int m = 0; m < npa; ++m)
        if (eidx[ep[e] + u * npa + m] != f0 + m)
          return set_err(c, CF_EINVAL, "enriched_tables: an atom's functions are not consecutive");
      if (u && f0 / npa <= atoms[i].back())
        return set_err(c, CF_EINVAL, "enriched_tables: a cell's atoms are not ascending");
      atoms[i].push_back(f0 / npa);
    }
  }
  // shared table
  std::vector<double> tab;
  tab.insert(tab.end(), g->nodes, g->nodes + np1);
  tab.insert(tab.end(), g->gauss_x, g->gauss_x + ng);
  tab.insert(tab.end(), g->gauss_w, g->gauss_w + ng);
  for (int s = 0; s < nsh && c->n_e > 0; ++s) tab.push_back(g->shell_l[s]);
  for (int s = 0; s <= nsh && c->n_e > 0; ++s) tab.push_back(g->shell_term_ptr[s]);
  for (int k = 0; k < nterm; ++k) {
    tab.push_back(g->term_c[k]);
    tab.push_back(g->term_k[k]);
    tab.push_back(g->term_zeta[k]);
  }
  // Work items.  A slot with more than EA_QCHUNK points is cut into point
  // chunks: its items write partial tiles, and a finishing group sums them in
  // chunk order.  Items are ordered by decreasing work (points times tiles)
  // so that the longest workgroups start first.
  const int64_t ng3q = (int64_t)ng * ng * ng;
  auto npts = [&](int64_t s) { return (g->box_ptr[s + 1] - g->box_ptr[s]) * ng3q; };
  // H^cc items
  std::vector<int32_t> nn_slot, nn_q0, nn_qn, nn_pi, nnf_slot, nnf_p0, nnf_np;
  {
    std::vector<std::array<int64_t, 5>> its;      // work, slot, q0, qn, pi
    int32_t np_nn = 0;
    for (int64_t s = 0; s < ncl; ++s) {
      const int64_t q = npts(s);
      if (q <= EA_QCHUNK) {
        its.push_back({q, s, 0, q, -1});
        continue;
      }
      nnf_slot.push_back((int32_t)s);
      nnf_p0.push_back(np_nn);
      for (int64_t q0 = 0; q0 < q; q0 += EA_QCHUNK) {
        const int64_t qn = std::min<int64_t>(EA_QCHUNK, q - q0);
        its.push_back({qn, s, q0, qn, np_nn++});
      }
      nnf_np.push_back(np_nn - nnf_p0.back());
    }
    std::stable_sort(its.begin(), its.end(), [](const std::array<int64_t, 5> &x,
                                                const std::array<int64_t, 5> &y) { return x[0] > y[0]; });
    for (const auto &x : its) {
      nn_slot.push_back((int32_t)x[1]);
      nn_q0.push_back((int32_t)x[2]);
      nn_qn.push_back((int32_t)x[3]);
      nn_pi.push_back((int32_t)x[4]);
    }
  }
  // enrichment-row items, their finishing groups and the atom-pair lists,
  // in batches of cells whose partial H^ee blocks fit EA_PEE_BYTES
  std::vector<int32_t> it_slot, it_t0, it_nt, it_q0, it_qn, it_pi, pair_ij, pc;
  std::vector<int32_t> f_slot, f_t0, f_nt, f_p0, f_np;
  std::vector<int64_t> pee_off(ncl, 0), pair_ptr(1, 0);
  std::vector<int> b_item(1, 0), b_pair(1, 0), b_fin(1, 0);
  int64_t pee_max = 0, ptile_max = 0;
  {
    int64_t used = 0;
    int32_t np_b = 0;                                // partial index within the batch
    std::vector<std::array<int64_t, 7>> its;         // work, slot, t0, nt, q0, qn, pi
    std::vector<int64_t> batch_slots;
    auto close_batch = [&]() {
      if (batch_slots.empty()) return;
      // pairs (I <= J) of each cell's atoms, cells in slot order
      std::vector<std::array<int32_t, 5>> ent;
      for (int64_t s : batch_slots)
        for (size_t u1 = 0; u1 < atoms[s].size(); ++u1)
          for (size_t u2 = u1; u2 < atoms[s].size(); ++u2)
            ent.push_back({atoms[s][u1], atoms[s][u2], (int32_t)s, (int32_t)u1, (int32_t)u2});
      std::stable_sort(ent.begin(), ent.end(), [](const std::array<int32_t, 5> &x,
                                                  const std::array<int32_t, 5> &y) {
        return x[0] != y[0] ? x[0] < y[0] : x[1] < y[1];
      });
      for (size_t q = 0; q < ent.size(); ++q) {
        if (q == 0 || ent[q][0] != ent[q - 1][0] || ent[q][1] != ent[q - 1][1]) {
          if (q) pair_ptr.push_back((int64_t)pc.size() / 3);
          pair_ij.push_back(ent[q][0]);
          pair_ij.push_back(ent[q][1]);
        }
        pc.push_back(ent[q][2]);
        pc.push_back(ent[q][3]);
        pc.push_back(ent[q][4]);
      }
      if (!ent.empty()) pair_ptr.push_back((int64_t)pc.size() / 3);
      std::stable_sort(its.begin(), its.end(), [](const std::array<int64_t, 7> &x,
                                                  const std::array<int64_t, 7> &y) { return x[0] > y[0]; });
      for (const auto &x : its) {
        it_slot.push_back((int32_t)x[1]);
        it_t0.push_back((int32_t)x[2]);
        it_nt.push_back((int32_t)x[3]);
        it_q0.push_back((int32_t)x[4]);
        it_qn.push_back((int32_t)x[5]);
        it_pi.push_back((int32_t)x[6]);
      }
      its.clear();
      b_item.push_back((int)it_slot.size());
      b_pair.push_back((int)pair_ij.size() / 2);
      b_fin.push_back((int)f_slot.size());
      pee_max = std::max(pee_max, used);
      ptile_max = std::max<int64_t>(ptile_max, np_b);
      batch_slots.clear();
      used = 0;
      np_b = 0;
    };
    for (int64_t s = 0; s < ncl; ++s) {
      if (atoms[s].empty()) continue;
      const int nap = (int)((atoms[s].size() * npa + 15) & ~(size_t)15), nte = nap / 16;
      const int64_t bytes = (int64_t)nap * nap * (int64_t)sizeof(double);
      if (used + bytes > EA_PEE_BYTES) close_batch();
      pee_off[s] = used / (int64_t)sizeof(double);
      used += bytes;
      batch_slots.push_back(s);
      const int ntiles = 8 * nte + nte * (nte + 1) / 2;
      const int64_t q = npts(s);
      for (int t0 = 0; t0 < ntiles; t0 += 4 * EA_TPW) {
        const int nt = std::min(4 * EA_TPW, ntiles - t0);
        if (q <= EA_QCHUNK) {
          its.push_back({q * nt, s, t0, nt, 0, q, -1});
          continue;
        }
        f_slot.push_back((int32_t)s);
        f_t0.push_back(t0);
        f_nt.push_back(nt);
        f_p0.push_back(np_b);
        for (int64_t q0 = 0; q0 < q; q0 += EA_QCHUNK) {
          const int64_t qn = std::min<int64_t>(EA_QCHUNK, q - q0);
          its.push_back({qn * nt, s, t0, nt, q0, qn, np_b++});
        }
        f_np.push_back(np_b - f_p0.back());
      }
    }
    close_batch();
  }
  // upload
  std::vector<double> lo(g->cell_lo, g->cell_lo + 3 * ncl);
  auto &ea = c->ea;
  STCHK(dupload(c, ea.cell, g->cells, (size_t)ncl));
  STCHK(dupload(c, ea.lo, lo.data(), lo.size()));
  STCHK(dupload(c, ea.bptr, g->box_ptr, (size_t)ncl + 1));
  STCHK(dupload(c, ea.blo, g->box_lo, (size_t)nbox * 3));
  STCHK(dupload(c, ea.bsz, g->box_size, (size_t)nbox));
  STCHK(dupload(c, ea.tab, tab.data(), tab.size()));
  if (c->n_e > 0) STCHK(dupload(c, ea.centers, g->centers, (size_t)g->n_atoms * 3));
  STCHK(dupload(c, ea.pee_off, pee_off.data(), pee_off.size()));
  STCHK(dupload(c, ea.item_slot, it_slot.data(), it_slot.size()));
  STCHK(dupload(c, ea.item_t0, it_t0.data(), it_t0.size()));
  STCHK(dupload(c, ea.item_nt, it_nt.data(), it_nt.size()));
  STCHK(dupload(c, ea.item_q0, it_q0.data(), it_q0.size()));
  STCHK(dupload(c, ea.item_qn, it_qn.data(), it_qn.size()));
  STCHK(dupload(c, ea.item_pi, it_pi.data(), it_pi.size()));
  STCHK(dupload(c, ea.f_slot, f_slot.data(), f_slot.size()));
  STCHK(dupload(c, ea.f_t0, f_t0.data(), f_t0.size()));
  STCHK(dupload(c, ea.f_nt, f_nt.data(), f_nt.size()));
  STCHK(dupload(c, ea.f_p0, f_p0.data(), f_p0.size()));
  STCHK(dupload(c, ea.f_np, f_np.data(), f_np.size()));
  STCHK(dupload(c, ea.nn_slot, nn_slot.data(), nn_slot.size()));
  STCHK(dupload(c, ea.nn_q0, nn_q0.data(), nn_q0.size()));
  STCHK(dupload(c, ea.nn_qn, nn_qn.data(), nn_qn.size()));
  STCHK(dupload(c, ea.nn_pi, nn_pi.data(), nn_pi.size()));
  STCHK(dupload(c, ea.nnf_slot, nnf_slot.data(), nnf_slot.size()));
  STCHK(dupload(c, ea.nnf_p0, nnf_p0.data(), nnf_p0.size()));
  STCHK(dupload(c, ea.nnf_np, nnf_np.data(), nnf_np.size()));
  dfree(c, ea.Ptile);
  STCHK(dalloc(c, &ea.Ptile, (size_t)std::max<int64_t>(ptile_max, 1) * 4 * EA_TPW * 256));
  dfree(c, ea.Pnn);
  STCHK(dalloc(c, &ea.Pnn, (size_t)std::max<size_t>(nn_pi.empty() ? 1 : (size_t)(1 + *std::max_element(nn_pi.begin(), nn_pi.end())), 1) * 36 * 256));
  ea.n_nn = (int)nn_slot.size();
  ea.n_nnf = (int)nnf_slot.size();
  ea.batch_fin = b_fin;
  STCHK(dupload(c, ea.pair_ij, pair_ij.data(), pair_ij.size()));
  STCHK(dupload(c, ea.pair_ptr, pair_ptr.data(), pair_ptr.size()));
  STCHK(dupload(c, ea.pc, pc.data(), pc.size()));
  dfree(c, ea.Pee);
  STCHK(dalloc(c, &ea.Pee, (size_t)std::max<int64_t>(pee_max / (int64_t)sizeof(double), 1)));
  ea.ncl = (int)ncl;
  ea.np1 = np1;
  ea.ng = ng;
  ea.nsh = c->n_e > 0 ? nsh : 0;
  ea.nterm = nterm;
  ea.npa = npa;
  ea.nbox = nbox;
  ea.npts = nbox * ng3;
  ea.h = g->h;
  ea.r0 = g->r0;
  ea.t = g->t;
  ea.batch_item = b_item;
  ea.batch_pair = b_pair;
  return CF_OK;
}

cf_status chebfilter_adaptive_points(const cf_ctx *c, int64_t *npoints) {
  if (!c || !npoints) return CF_EINVAL;
  *npoints = c->ea.npts;
  return CF_OK;
}

// Hmod = H^ee - M^ec D^-1 H^ec^T (the enrichment block of H~'s step, Sec. IV.D)
// from the current coupling blocks, ldw unit columns at a time: the
// transposed coupling products of the unit block gathered and scaled by D^-1
// on the enriched region's classical rows, then the M^ec partial products of
// that block and their fixed-order sums, subtracted from the columns of H^ee.
static cf_status rebuild_hmod(cf_ctx *c) {
  const int64_t n_e = c->n_e, lw = c->ldw;
  HIPCHK(c, launch_fill(c->stream, c->T, c->n * lw, 0.0));
  for (int64_t j0 = 0; j0 < n_e; j0 += lw) {
    const int nb = (int)std::min<int64_t>(lw, n_e - j0);
    HIPCHK(c, launch_unit_cols(c->stream, n_e, nb, lw, j0, c->Wb));
    STCHK(core_enr_q(c, c->Wb, lw, 1.0, nullptr, 0, 0.0, nb));
    EpiArgs g = epi_base(c, nb);
    g.rows = c->regrows;
    g.nrows = c->nregrows;
    g.R = c->T; g.ldr = lw;
    g.dC = c->dinv;
    g.Ee = c->Wb; g.lde = lw;
    g.Out = c->U; g.ldo = lw;
    HIPCHK(c, launch_epilogue(c->stream, g));
    HIPCHK(c, launch_enr_part(c->stream, c->HT, c->MT, c->toff, c->tld, c->eptr, c->dofp,
                              c->ecells_part, c->necells, c->epitems, c->nepitems, nullptr, 0, 0.0,
                              c->U, lw, nullptr, 1.0,
                              c->P, lw, nb));
    HIPCHK(c, launch_enr_reduce(c->stream, (int)n_e, c->aptr, c->alist, c->P, lw, -1.0,
                                c->Hee + j0, n_e, 1.0, nullptr, nullptr, 0, c->Hmod + j0, n_e, nb));
  }
  return CF_OK;
}

cf_status chebfilter_assemble_enriched(cf_ctx *c, const double *V) {
  if (!c) return CF_EINVAL;
  auto &ea = c->ea;
  if (ea.ncl == 0) return set_err(c, CF_EINVAL, "assemble_enriched: no grid (chebfilter_enriched_tables)");
  if (!V) return set_err(c, CF_EINVAL, "assemble_enriched: null potential");
  HIPCHK(c, hipSetDevice(c->device));
  EnrAsm a;
  a.ncl = ea.ncl;
  a.cell = ea.cell; a.lo = ea.lo; a.bptr = ea.bptr; a.blo = ea.blo; a.bsz = ea.bsz; a.V = V;
  a.ng = ea.ng; a.np1 = ea.np1; a.h = ea.h; a.tab = ea.tab;
  a.nsh = ea.nsh; a.nterm = ea.nterm; a.npa = ea.npa; a.r0 = ea.r0; a.t = ea.t;
  a.centers = ea.centers;
  a.eptr = c->eptr; a.eidx = c->eidx; a.tld = c->tld; a.toff = c->toff;
  a.Hp = c->Hp; a.K = c->asm_K; a.Hec = c->Hec; a.HT = c->HT;
  a.Pee = ea.Pee; a.pee_off = ea.pee_off;
  a.Ptile = ea.Ptile; a.Pnn = ea.Pnn;
  a.nn_slot = ea.nn_slot; a.nn_q0 = ea.nn_q0; a.nn_qn = ea.nn_qn; a.nn_pi = ea.nn_pi;
  a.nnf_slot = ea.nnf_slot; a.nnf_p0 = ea.nnf_p0; a.nnf_np = ea.nnf_np;
  {
    Scope sc(c, "assemble_adaptive");
    HIPCHK(c, launch_ea_nn(c->stream, a, ea.n_nn, ea.n_nnf));
    if (c->n_e > 0) {
      HIPCHK(c, launch_fill(c->stream, c->Hee, c->n_e * c->n_e, 0.0));
      for (size_t b = 0; b + 1 < ea.batch_item.size(); ++b) {
        EnrAsm ab = a;
        const int i0 = ea.batch_item[b], f0 = ea.batch_fin[b];
        ab.item_slot = ea.item_slot + i0;
        ab.item_t0 = ea.item_t0 + i0;
        ab.item_nt = ea.item_nt + i0;
        ab.item_q0 = ea.item_q0 + i0;
        ab.item_qn = ea.item_qn + i0;
        ab.item_pi = ea.item_pi + i0;
        ab.fin_slot = ea.f_slot + f0;
        ab.fin_t0 = ea.f_t0 + f0;
        ab.fin_nt = ea.f_nt + f0;
        ab.fin_p0 = ea.f_p0 + f0;
        ab.fin_np = ea.f_np + f0;
        HIPCHK(c, launch_ea_erow(c->stream, ab, ea.batch_item[b + 1] - i0, ea.batch_fin[b + 1] - f0));
        HIPCHK(c, launch_ea_ee_reduce(c->stream, a, (int)c->n_e,
                                      ea.batch_pair[b + 1] - ea.batch_pair[b],
                                      ea.pair_ij + 2 * (int64_t)ea.batch_pair[b],
                                      ea.pair_ptr + ea.batch_pair[b], ea.pc, c->Hee));
      }
    }
  }
  if (c->n_e > 0) {
    Scope sc(c, "rebuild_hmod");
    STCHK(rebuild_hmod(c));
  }
  const int64_t hsz = c->E * NPAD * NPAD;
  if (c->Hp32) HIPCHK(c, launch_to_f32(c->stream, hsz, c->Hp, c->Hp32));
  if (c->Hp16) HIPCHK(c, launch_to_bf16(c->stream, hsz, c->Hp, c->Hp16));
  if (c->HT32) HIPCHK(c, launch_to_f32(c->stream, c->ttot, c->HT, c->HT32));
  if (c->Hec32) HIPCHK(c, launch_to_f32(c->stream, c->nnz * NPAD, c->Hec, c->Hec32));
  return CF_OK;
}

cf_status chebfilter_get_coupling(cf_ctx *c, double *H_ec, double *H_ee) {
  if (!c) return CF_EINVAL;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->n_e == 0) return CF_OK;
  const int npc = c->npc;
  if (H_ec) {
    const int64_t batch = 4096;
    std::vector<double> buf((size_t)batch * NPAD);
    for (int64_t k0 = 0; k0 < c->nnz; k0 += batch) {
      const int64_t nbk = std::min(batch, c->nnz - k0);
      HIPCHK(c, hipMemcpy(buf.data(), c->Hec + k0 * NPAD, nbk * NPAD * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t k = 0; k < nbk; ++k)
        for (int a2 = 0; a2 < npc; ++a2) H_ec[(k0 + k) * npc + a2] = buf[k * NPAD + a2];
    }
  }
  if (H_ee) HIPCHK(c, hipMemcpy(H_ee, c->Hee, c->n_e * c->n_e * sizeof(double), hipMemcpyDeviceToHost));
  return CF_OK;
}

// ---------------------------------------------------------------------------
// Self-consistent field quantities (Sec. II, Sec. V)
// ---------------------------------------------------------------------------
static constexpr int SCF_RED_BLOCKS = 1024;         // fixed grid of the weighted sums
static constexpr int SCF_CG_CHECK = 10;             // CG iterations between host checks
static constexpr int64_t SCF_DM_BYTES = 1ll << 30;  // density matrices of one batch

cf_status chebfilter_fermi_level(const double *eps, int64_t N, double n_electrons, double kT,
                                 double *f, double *mu) {
  if (!eps || !f || !mu || N < 1 || !(kT > 0.0) || !std::isfinite(kT)) return CF_EINVAL;
  if (!(n_electrons > 0.0) || !(n_electrons < 2.0 * (double)N)) return CF_EINVAL;
  double lo = eps[0], hi = eps[0];
  for (int64_t i = 0; i < N; ++i) {
    if (!std::isfinite(eps[i])) return CF_EINVAL;
    lo = std::min(lo, eps[i]);
    hi = std::max(hi, eps[i]);
  }
  lo -= 40.0 * kT;
  hi += 40.0 * kT;
  auto occ = [&](double m, int64_t i) {
    const double x = (eps[i] - m) / kT;
    if (x > 0.0) { const double ex = std::exp(-x); return ex / (1.0 + ex); }
    return 1.0 / (1.0 + std::exp(x));
  };
  for (int it = 0; it < 200; ++it) {
    const double m = 0.5 * (lo + hi);
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += occ(m, i);
    if (2.0 * s < n_electrons) lo = m; else hi = m;
    if (hi - lo <= 4e-16 * std::max(1.0, std::fabs(m))) break;
  }
  *mu = 0.5 * (lo + hi);
  for (int64_t i = 0; i < N; ++i) f[i] = occ(*mu, i);
  return CF_OK;
}

static ScfArgs scf_args(cf_ctx *c) {
  ScfArgs g;
  const auto &s = c->scf;
  g.n_h = c->n_h;
  g.np1 = c->ea.np1;
  g.ng = c->ea.ng;
  g.nsh = c->ea.nsh;
  g.npa = c->ea.npa;
  g.ntab = ea_tab_size(c->ea.np1, c->ea.ng, c->ea.nsh, c->ea.nterm);
  g.h = c->ea.h;
  g.r0 = c->ea.r0;
  g.t = c->ea.t;
  g.tab = c->ea.tab;
  g.centers = c->ea.centers;
  g.dofp = c->dofp;
  g.eptr = c->eptr;
  g.eidx = c->eidx;
  g.cell = s.cell;
  g.cna = s.cna;
  g.lo = s.lo;
  g.pofs = s.pofs;
  g.pcnt = s.pcnt;
  g.doff = s.doff;
  g.xyz = s.xyz;
  g.w = s.w;
  for (int d = 0; d < 3; ++d) g.cc[d] = s.cc[d];
  g.cs = s.cs;
  return g;
}

cf_status chebfilter_scf_setup(cf_ctx *c, const cf_scf_setup *o) {
  if (!c) return CF_EINVAL;
  if (!o || !o->cell_lo || !o->plain_ref) return set_err(c, CF_EINVAL, "scf_setup: null argument");
  if (!c->asm_K) return set_err(c, CF_EINVAL, "scf_setup: no plain rule (chebfilter_assembly_tables)");
  if (c->ea.ncl == 0) return set_err(c, CF_EINVAL, "scf_setup: no adaptive grid (chebfilter_enriched_tables)");
  if (!(o->comp_width > 0.0) || o->cg_max_iter < 1 || !(o->cg_tol > 0.0) || o->mix_depth < 1 ||
      o->mix_depth > 8 || !(o->mix_beta > 0.0))
    return set_err(c, CF_EINVAL, "scf_setup: bad width, CG limits or mixing depth (1..8) / beta");
  const int64_t E = c->E, nq = c->asm_nq;
  auto &s = c->scf;
  auto &ea = c->ea;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // host copies of what the device holds
  std::vector<int32_t> eacell(ea.ncl), dofp((size_t)E * NPAD), colcells(E);
  std::vector<int64_t> bptr(ea.ncl + 1), ep(E + 1, 0);
  std::vector<double> blo((size_t)ea.nbox * 3), bsz(ea.nbox), tab(ea_tab_size(ea.np1, ea.ng, ea.nsh, ea.nterm)),
      wq(nq), K((size_t)NPAD * NPAD);
  HIPCHK(c, hipMemcpy(eacell.data(), ea.cell, ea.ncl * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(dofp.data(), c->dofp, dofp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(colcells.data(), c->cells, E * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(bptr.data(), ea.bptr, bptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(blo.data(), ea.blo, blo.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(bsz.data(), ea.bsz, bsz.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(tab.data(), ea.tab, tab.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(wq.data(), c->asm_w, nq * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(c, hipMemcpy(K.data(), c->asm_K, K.size() * sizeof(double), hipMemcpyDeviceToHost));
  if (c->n_e > 0) HIPCHK(c, hipMemcpy(ep.data(), c->eptr, (E + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  for (int64_t q = 0; q < 3 * E; ++q)
    if (!std::isfinite(o->cell_lo[q])) return set_err(c, CF_EINVAL, "scf_setup: non-finite cell corner");
  for (int64_t q = 0; q < 3 * nq; ++q)
    if (!(o->plain_ref[q] >= 0.0 && o->plain_ref[q] <= 1.0))
      return set_err(c, CF_EINVAL, "scf_setup: plain rule points must lie in the unit cube");
  // SCF cells: the plain cells in index order, then the adaptive slots
  std::vector<uint8_t> listed(E, 0);
  for (int32_t e : eacell) listed[e] = 1;
  std::vector<int32_t> cell, cna;
  std::vector<int64_t> pofs, pcnt;
  std::vector<double> lo;
  s.plain_cells.clear();
  for (int64_t e = 0; e < E; ++e)
    if (!listed[e]) s.plain_cells.push_back((int32_t)e);
  const int64_t ng3 = (int64_t)ea.ng * ea.ng * ea.ng;
  int64_t P = 0;
  for (int32_t e : s.plain_cells) {
    cell.push_back(e);
    cna.push_back(0);
    pofs.push_back(P);
    pcnt.push_back(nq);
    P += nq;
  }
  const int64_t P_plain = P;
  for (int i = 0; i < ea.ncl; ++i) {
    const int32_t e = eacell[i];
    cell.push_back(e);
    cna.push_back(c->n_e > 0 ? (int32_t)(ep[e + 1] - ep[e]) : 0);
    pofs.push_back(P);
    pcnt.push_back((bptr[i + 1] - bptr[i]) * ng3);
    P += (bptr[i + 1] - bptr[i]) * ng3;
  }
  const int nscf = (int)cell.size();
  for (int32_t e : cell)
    for (int d = 0; d < 3; ++d) lo.push_back(o->cell_lo[3 * (int64_t)e + d]);
  // points and weights
  std::vector<double> xyz((size_t)P * 3), w(P);
  const double h = ea.h;
  for (size_t i = 0; i < s.plain_cells.size(); ++i) {
    const int32_t e = s.plain_cells[i];
    for (int64_t q = 0; q < nq; ++q) {
      const int64_t p = (int64_t)i * nq + q;
      for (int d = 0; d < 3; ++d) xyz[3 * p + d] = o->cell_lo[3 * (int64_t)e + d] + h * o->plain_ref[3 * q + d];
      w[p] = wq[q];
    }
  }
  const double *gx = tab.data() + ea.np1, *gw = gx + ea.ng;
  for (int64_t b = 0; b < ea.nbox; ++b)
    for (int64_t r = 0; r < ng3; ++r) {
      const int ix = (int)(r % ea.ng), iy = (int)((r / ea.ng) % ea.ng), iz = (int)(r / (ea.ng * ea.ng));
      const int64_t p = P_plain + b * ng3 + r;
      const double sd = bsz[b];
      xyz[3 * p] = blo[3 * b] + sd * gx[ix];
      xyz[3 * p + 1] = blo[3 * b + 1] + sd * gx[iy];
      xyz[3 * p + 2] = blo[3 * b + 2] + sd * gx[iz];
      w[p] = sd * sd * sd * (gw[ix] * gw[iy] * gw[iz]);
    }
  // density-matrix items (upper 16 x 16 tiles, at most 64 per item) in batches
  std::vector<int32_t> it_c, it_t0, it_nt;
  std::vector<int64_t> doff(nscf, 0);
  std::vector<int> b_item(1, 0), b_cell(1, 0);
  int64_t used = 0, dmax = 0;
  for (int i = 0; i < nscf; ++i) {
    const int K = NPAD + ((cna[i] + 15) & ~15), nt = K / 16;
    const int64_t bytes = (int64_t)K * K * (int64_t)sizeof(double);
    if (used && used + bytes > SCF_DM_BYTES) {
      b_item.push_back((int)it_c.size());
      b_cell.push_back(i);
      used = 0;
    }
    doff[i] = used / (int64_t)sizeof(double);
    used += bytes;
    dmax = std::max(dmax, used);
    const int ntiles = nt * (nt + 1) / 2;
    for (int t0 = 0; t0 < ntiles; t0 += 64) {
      it_c.push_back(i);
      it_t0.push_back(t0);
      it_nt.push_back(std::min(64, ntiles - t0));
    }
  }
  b_item.push_back((int)it_c.size());
  b_cell.push_back(nscf);
  // density items per batch and range index r: the upper tiles
  // [r SCF_RHO_TILES, (r + 1) SCF_RHO_TILES) of every cell that has them; the
  // items of range 0 write rho, each later range adds in a launch of its own
  // (so that one launch never holds two items of one cell)
  // Each range's items are cut into chunks of at most SCF_RHO_QCHUNK points
  // and ordered by decreasing work (points times tiles), so that the longest
  // start first.
  std::vector<int32_t> r_c, r_t0, r_nt, r_q0;
  std::vector<int> r_off;
  const int nrange = (ea_max_tiles(NPAD + EA_MAXNAP) + SCF_RHO_TILES - 1) / SCF_RHO_TILES;
  for (size_t b = 0; b + 1 < b_cell.size(); ++b)
    for (int r = 0; r < nrange; ++r) {
      r_off.push_back((int)r_c.size());
      std::vector<std::array<int64_t, 5>> its;   // work, cell, t0, nt, q0
      for (int i = b_cell[b]; i < b_cell[b + 1]; ++i) {
        const int K = NPAD + ((cna[i] + 15) & ~15), ntiles = ea_max_tiles(K);
        const int t0 = r * SCF_RHO_TILES;
        if (t0 >= ntiles) continue;
        const int nt = std::min(SCF_RHO_TILES, ntiles - t0);
        for (int64_t q0 = 0; q0 < pcnt[i]; q0 += SCF_RHO_QCHUNK)
          its.push_back({std::min<int64_t>(SCF_RHO_QCHUNK, pcnt[i] - q0) * (nt + 32), i, t0, nt, q0});
      }
      std::stable_sort(its.begin(), its.end(), [](const std::array<int64_t, 5> &x,
                                                  const std::array<int64_t, 5> &y) {
        return x[0] > y[0];
      });
      for (const auto &x : its) {
        r_c.push_back((int32_t)x[1]);
        r_t0.push_back((int32_t)x[2]);
        r_nt.push_back((int32_t)x[3]);
        r_q0.push_back((int32_t)x[4]);
      }
    }
  r_off.push_back((int)r_c.size());
  // per colour, the SCF cells of that colour
  std::vector<int32_t> scf_of(E, -1), colscf;
  for (int i = 0; i < nscf; ++i) scf_of[cell[i]] = i;
  std::vector<int> cofs(1, 0);
  for (size_t k = 0; k + 1 < c->col_off.size(); ++k) {
    const size_t b0 = colscf.size();
    for (int q = c->col_off[k]; q < c->col_off[k + 1]; ++q) colscf.push_back(scf_of[colcells[q]]);
    // the cells with the most points first (the longest workgroups start first)
    std::stable_sort(colscf.begin() + b0, colscf.end(),
                     [&](int32_t x, int32_t y) { return pcnt[x] > pcnt[y]; });
    cofs.push_back((int)colscf.size());
  }
  // Poisson: A^C block = K / (2 pi) (K = 1/2 int grad N . grad N), Jacobi diagonal
  std::vector<double> A(K.size()), diag(c->n_h, 0.0);
  for (size_t q = 0; q < K.size(); ++q) A[q] = K[q] / (2.0 * M_PI);
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < NPAD; ++a) {
      const int32_t d = dofp[e * NPAD + a];
      if (d >= 0) diag[d] += A[(size_t)a * NPAD + a];
    }
  for (auto &x : diag) {
    if (!(x > 0.0)) return set_err(c, CF_EINVAL, "scf_setup: non-positive Laplace diagonal");
    x = 1.0 / x;
  }
  std::vector<int32_t> seq(nscf);
  for (int i = 0; i < nscf; ++i) seq[i] = i;
  STCHK(dupload(c, s.cell, cell.data(), cell.size()));
  STCHK(dupload(c, s.cna, cna.data(), cna.size()));
  STCHK(dupload(c, s.seq, seq.data(), seq.size()));
  STCHK(dupload(c, s.col_cells, colscf.data(), colscf.size()));
  STCHK(dupload(c, s.dm_c, it_c.data(), it_c.size()));
  STCHK(dupload(c, s.dm_t0, it_t0.data(), it_t0.size()));
  STCHK(dupload(c, s.dm_nt, it_nt.data(), it_nt.size()));
  STCHK(dupload(c, s.rho_c, r_c.data(), r_c.size()));
  STCHK(dupload(c, s.rho_t0, r_t0.data(), r_t0.size()));
  STCHK(dupload(c, s.rho_nt, r_nt.data(), r_nt.size()));
  STCHK(dupload(c, s.rho_q0, r_q0.data(), r_q0.size()));
  s.rho_off = r_off;
  STCHK(dupload(c, s.pofs, pofs.data(), pofs.size()));
  STCHK(dupload(c, s.pcnt, pcnt.data(), pcnt.size()));
  STCHK(dupload(c, s.doff, doff.data(), doff.size()));
  STCHK(dupload(c, s.lo, lo.data(), lo.size()));
  STCHK(dupload(c, s.xyz, xyz.data(), xyz.size()));
  STCHK(dupload(c, s.w, w.data(), w.size()));
  STCHK(dupload(c, s.A, A.data(), A.size()));
  STCHK(dupload(c, s.dinv, diag.data(), diag.size()));
  dfree(c, s.Dbuf);
  STCHK(dalloc(c, &s.Dbuf, (size_t)std::max<int64_t>(dmax / (int64_t)sizeof(double), 1)));
  for (double **v : {&s.pb, &s.px, &s.pr, &s.pz, &s.pp, &s.pq}) {
    dfree(c, *v);
    STCHK(dalloc(c, v, (size_t)std::max<int64_t>(c->n_h, 1)));
  }
  HIPCHK(c, launch_fill(c->stream, s.px, c->n_h, 0.0));
  dfree(c, s.vxc);
  STCHK(dalloc(c, &s.vxc, (size_t)std::max<int64_t>(P, 1)));
  dfree(c, s.part);
  STCHK(dalloc(c, &s.part, (size_t)std::max<int64_t>(4 * SCF_RED_BLOCKS, nscf)));
  dfree(c, s.dot);
  STCHK(dalloc(c, &s.dot, (size_t)SCF_RED_BLOCKS + 8));
  dfree(c, s.hin);
  dfree(c, s.hF);
  STCHK(dalloc(c, &s.hin, (size_t)std::max<int64_t>(P, 1) * o->mix_depth));
  STCHK(dalloc(c, &s.hF, (size_t)std::max<int64_t>(P, 1) * o->mix_depth));
  s.nscf = nscf;
  s.nplain = (int)s.plain_cells.size();
  s.nq = (int)nq;
  s.P = P;
  s.P_plain = P_plain;
  for (int d = 0; d < 3; ++d) s.cc[d] = o->comp_center[d];
  s.cs = o->comp_width;
  s.cg_max = o->cg_max_iter;
  s.cg_tol = o->cg_tol;
  s.depth = o->mix_depth;
  s.beta = o->mix_beta;
  s.nhist = s.head = 0;
  s.gram.assign((size_t)o->mix_depth * o->mix_depth, 0.0);
  s.dm_item = b_item;
  s.dm_cell = b_cell;
  s.col_ofs = cofs;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CF_OK;
}

cf_status chebfilter_scf_sizes(const cf_ctx *c, int64_t *npoints, int64_t *nplain_points) {
  if (!c) return CF_EINVAL;
  if (npoints) *npoints = c->scf.P;
  if (nplain_points) *nplain_points = c->scf.P_plain;
  return CF_OK;
}

cf_status chebfilter_scf_geometry(cf_ctx *c, double *xyz, double *w) {
  if (!c) return CF_EINVAL;
  if (c->scf.P == 0) return set_err(c, CF_EINVAL, "scf_geometry: no SCF setup");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (xyz) HIPCHK(c, hipMemcpy(xyz, c->scf.xyz, c->scf.P * 3 * sizeof(double), hipMemcpyDeviceToHost));
  if (w) HIPCHK(c, hipMemcpy(w, c->scf.w, c->scf.P * sizeof(double), hipMemcpyDeviceToHost));
  return CF_OK;
}

cf_status chebfilter_scf_density(cf_ctx *c, const double *X, int64_t ldx, int64_t N,
                                 const double *f_host, double *rho) {
  if (!c) return CF_EINVAL;
  auto &s = c->scf;
  if (s.P == 0) return set_err(c, CF_EINVAL, "scf_density: no SCF setup");
  if (!X || !f_host || !rho || N < 1 || ldx < N) return set_err(c, CF_EINVAL, "scf_density: bad block");
  for (int64_t j = 0; j < N; ++j)
    if (!std::isfinite(f_host[j])) return set_err(c, CF_EINVAL, "scf_density: non-finite occupation");
  HIPCHK(c, hipSetDevice(c->device));
  if (N > s.f2_cap) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, s.f2);
    STCHK(dalloc(c, &s.f2, (size_t)N));
    s.f2_cap = N;
  }
  std::vector<double> f2(N);
  for (int64_t j = 0; j < N; ++j) f2[j] = 2.0 * f_host[j];
  HIPCHK(c, hipMemcpyAsync(s.f2, f2.data(), N * sizeof(double), hipMemcpyHostToDevice, c->stream));
  const ScfArgs g = scf_args(c);
  Scope sc(c, "scf_density");
  for (size_t b = 0; b + 1 < s.dm_item.size(); ++b) {
    HIPCHK(c, launch_scf_dm(c->stream, g, s.dm_item[b + 1] - s.dm_item[b], s.dm_c + s.dm_item[b],
                            s.dm_t0 + s.dm_item[b], s.dm_nt + s.dm_item[b], X, ldx, (int)N, s.f2,
                            s.Dbuf));
    const int nrange = (int)(s.rho_off.size() - 1) / (int)(s.dm_item.size() - 1);
    for (int r = 0; r < nrange; ++r) {
      const int i0 = s.rho_off[b * nrange + r], i1 = s.rho_off[b * nrange + r + 1];
      HIPCHK(c, launch_scf_rho(c->stream, g, i1 - i0, s.rho_c + i0, s.rho_t0 + i0, s.rho_nt + i0,
                               s.rho_q0 + i0, r > 0, s.Dbuf, rho));
    }
  }
  // the host copy of f2 must outlive the asynchronous copy
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CF_OK;
}

static cf_status scf_dot(cf_ctx *c, const double *x, const double *y, int64_t n, double *out) {
  HIPCHK(c, launch_dot(c->stream, n, x, y, c->scf.dot + SCF_RED_BLOCKS, c->scf.dot, SCF_RED_BLOCKS));
  HIPCHK(c, hipMemcpyAsync(out, c->scf.dot + SCF_RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return CF_OK;
}

// y = A x over all colours (y zeroed first)
static cf_status scf_lap(cf_ctx *c, const ScfArgs &g, const double *x, double *y) {
  auto &s = c->scf;
  HIPCHK(c, launch_fill(c->stream, y, c->n_h, 0.0));
  for (size_t k = 0; k + 1 < s.col_ofs.size(); ++k)
    HIPCHK(c, launch_scf_lap(c->stream, g, s.col_ofs[k + 1] - s.col_ofs[k], s.col_cells + s.col_ofs[k],
                             s.A, x, y));
  return CF_OK;
}

cf_status chebfilter_scf_potential(cf_ctx *c, const double *rho, const double *v_ext, double *v_eff,
                                   double *terms, int32_t *cg_iters) {
  if (!c) return CF_EINVAL;
  auto &s = c->scf;
  if (s.P == 0) return set_err(c, CF_EINVAL, "scf_potential: no SCF setup");
  if (!rho || !v_ext || !v_eff || !terms) return set_err(c, CF_EINVAL, "scf_potential: null argument");
  HIPCHK(c, hipSetDevice(c->device));
  ScfArgs g = scf_args(c);
  Scope sc(c, "scf_potential");
  // LDA and the charge
  std::vector<double> part(4 * SCF_RED_BLOCKS);
  HIPCHK(c, launch_scf_lda(c->stream, s.P, rho, s.w, s.vxc, s.part, SCF_RED_BLOCKS));
  HIPCHK(c, hipMemcpyAsync(part.data(), s.part, part.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double Q = 0.0, Exc = 0.0, Vxc = 0.0;
  for (int b = 0; b < SCF_RED_BLOCKS; ++b) {
    Q += part[4 * b];
    Exc += part[4 * b + 1];
    Vxc += part[4 * b + 2];
  }
  g.Q = Q;
  // right-hand side of the neutralised density, colour by colour
  HIPCHK(c, launch_fill(c->stream, s.pb, c->n_h, 0.0));
  for (size_t k = 0; k + 1 < s.col_ofs.size(); ++k)
    HIPCHK(c, launch_scf_rhs(c->stream, g, s.col_ofs[k + 1] - s.col_ofs[k], s.col_cells + s.col_ofs[k],
                             rho, s.pb));
  // Jacobi-preconditioned CG from the previous solution
  double bb = 0.0;
  STCHK(scf_dot(c, s.pb, s.pb, c->n_h, &bb));
  // r = b - A x0 (q = A x0)
  STCHK(scf_lap(c, g, s.px, s.pq));
  HIPCHK(c, launch_scf_cg(c->stream, c->n_h, 3, 0.0, 0.0, nullptr, nullptr, s.pr, s.pb, nullptr, s.pq));
  // the scalars stay on the device (s.dot[SCF_RED_BLOCKS + 1 ..]); the host
  // reads r.r every SCF_CG_CHECK iterations to stop
  double *dsc = s.dot + SCF_RED_BLOCKS + 1;
  int it = 0;
  double rr = 0.0;
  HIPCHK(c, launch_dot(c->stream, c->n_h, s.pr, s.pr, dsc + 2, s.dot, SCF_RED_BLOCKS));
  HIPCHK(c, hipMemcpyAsync(&rr, dsc + 2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double stop = s.cg_tol * s.cg_tol * std::max(bb, 1e-300);
  if (rr > stop) {
    HIPCHK(c, launch_scf_cg(c->stream, c->n_h, 0, 0.0, 0.0, s.dinv, nullptr, s.pr, s.pz, nullptr, nullptr));
    HIPCHK(c, launch_copy(c->stream, c->n_h, 1, s.pz, 1, s.pp, 1));
    HIPCHK(c, launch_dot(c->stream, c->n_h, s.pr, s.pz, dsc + 0, s.dot, SCF_RED_BLOCKS));
    for (it = 1; it <= s.cg_max; ++it) {
      STCHK(scf_lap(c, g, s.pp, s.pq));
      HIPCHK(c, launch_dot(c->stream, c->n_h, s.pp, s.pq, dsc + 1, s.dot, SCF_RED_BLOCKS));
      HIPCHK(c, launch_scf_cgd(c->stream, c->n_h, 0, dsc, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));
      HIPCHK(c, launch_scf_cgd(c->stream, c->n_h, 1, dsc, s.dinv, s.px, s.pr, s.pz, s.pp, s.pq));
      HIPCHK(c, launch_dot(c->stream, c->n_h, s.pr, s.pz, dsc + 3, s.dot, SCF_RED_BLOCKS));
      HIPCHK(c, launch_scf_cgd(c->stream, c->n_h, 2, dsc, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));
      HIPCHK(c, launch_scf_cgd(c->stream, c->n_h, 3, dsc, nullptr, nullptr, nullptr, s.pz, s.pp, nullptr));
      if (it % SCF_CG_CHECK == 0 || it == s.cg_max) {
        HIPCHK(c, launch_dot(c->stream, c->n_h, s.pr, s.pr, dsc + 2, s.dot, SCF_RED_BLOCKS));
        double scal[2] = {0.0, 0.0};
        HIPCHK(c, hipMemcpyAsync(scal, dsc + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (!(scal[0] > 0.0)) return set_err(c, CF_EDEVICE, "scf_potential: CG lost positive definiteness");
        rr = scal[1];
        if (rr <= stop) break;
      }
    }
  }
  if (cg_iters) *cg_iters = it;
  if (rr > stop) return set_err(c, CF_ENOTCONV, "scf_potential: CG did not reach the tolerance");
  // V_H and V_eff at the points, and sum w rho V_H per SCF cell
  HIPCHK(c, launch_scf_veff(c->stream, g, s.nscf, s.px, rho, v_ext, s.vxc, v_eff, s.part));
  std::vector<double> pc(s.nscf);
  HIPCHK(c, hipMemcpyAsync(pc.data(), s.part, s.nscf * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double EH = 0.0;
  for (double x : pc) EH += x;
  terms[0] = Q;
  terms[1] = Exc;
  terms[2] = Vxc;
  terms[3] = 0.5 * EH;
  terms[4] = std::sqrt(rr / std::max(bb, 1e-300));
  return CF_OK;
}

cf_status chebfilter_scf_assemble(cf_ctx *c, const double *v_eff) {
  if (!c) return CF_EINVAL;
  auto &s = c->scf;
  if (s.P == 0) return set_err(c, CF_EINVAL, "scf_assemble: no SCF setup");
  if (!v_eff) return set_err(c, CF_EINVAL, "scf_assemble: null potential");
  if (s.nplain > 0)
    STCHK(chebfilter_assemble_cells(c, s.plain_cells.data(), s.nplain, v_eff, s.nq));
  return chebfilter_assemble_enriched(c, v_eff + s.P_plain);
}

static cf_status scf_wdot(cf_ctx *c, const double *a, const double *b, double *out) {
  auto &s = c->scf;
  std::vector<double> part(SCF_RED_BLOCKS);
  HIPCHK(c, launch_scf_wdot(c->stream, s.P, s.w, a, b, s.part, SCF_RED_BLOCKS));
  HIPCHK(c, hipMemcpyAsync(part.data(), s.part, SCF_RED_BLOCKS * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double v = 0.0;
  for (double x : part) v += x;
  *out = v;
  return CF_OK;
}

cf_status chebfilter_scf_mix(cf_ctx *c, const double *rho_in, const double *rho_out, double *rho_next,
                             double *res_norm) {
  if (!c) return CF_EINVAL;
  auto &s = c->scf;
  if (s.P == 0) return set_err(c, CF_EINVAL, "scf_mix: no SCF setup");
  if (!rho_in || !rho_out || !rho_next) return set_err(c, CF_EINVAL, "scf_mix: null argument");
  HIPCHK(c, hipSetDevice(c->device));
  const int slot = s.head, D = s.depth;
  HIPCHK(c, launch_scf_push(c->stream, s.P, rho_in, rho_out, s.hin + (int64_t)slot * s.P,
                            s.hF + (int64_t)slot * s.P));
  s.nhist = std::min(s.nhist + 1, D);
  s.head = (s.head + 1) % D;
  for (int k = 0; k < s.nhist; ++k) {
    double v = 0.0;
    STCHK(scf_wdot(c, s.hF + (int64_t)slot * s.P, s.hF + (int64_t)k * s.P, &v));
    s.gram[(size_t)slot * D + k] = v;
    s.gram[(size_t)k * D + slot] = v;
  }
  if (res_norm) *res_norm = std::sqrt(std::max(s.gram[(size_t)slot * D + slot], 0.0));
  // [G 1; 1^T 0] [c; lambda] = [0; 1] by Gaussian elimination with partial pivoting
  const int m = s.nhist, n = m + 1;
  std::vector<double> M((size_t)n * (n + 1), 0.0);
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) M[(size_t)i * (n + 1) + j] = s.gram[(size_t)i * D + j];
    M[(size_t)i * (n + 1) + m] = 1.0;
    M[(size_t)m * (n + 1) + i] = 1.0;
  }
  M[(size_t)m * (n + 1) + n] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * (n + 1) + col]) > std::fabs(M[(size_t)piv * (n + 1) + col])) piv = r;
    if (M[(size_t)piv * (n + 1) + col] == 0.0) return set_err(c, CF_EINVAL, "scf_mix: singular history");
    if (piv != col)
      for (int j = 0; j <= n; ++j) std::swap(M[(size_t)piv * (n + 1) + j], M[(size_t)col * (n + 1) + j]);
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = M[(size_t)r * (n + 1) + col] / M[(size_t)col * (n + 1) + col];
      if (f == 0.0) continue;
      for (int j = col; j <= n; ++j) M[(size_t)r * (n + 1) + j] -= f * M[(size_t)col * (n + 1) + j];
    }
  }
  ScfMixCoef cf;
  for (int k = 0; k < 8; ++k) cf.c[k] = 0.0;
  for (int k = 0; k < m; ++k) cf.c[k] = M[(size_t)k * (n + 1) + n] / M[(size_t)k * (n + 1) + k];
  HIPCHK(c, launch_scf_mix(c->stream, s.P, m, cf, s.beta, s.hin, s.hF, s.P, rho_next));
  return CF_OK;
}

cf_status chebfilter_scf_mix_reset(cf_ctx *c) {
  if (!c) return CF_EINVAL;
  c->scf.nhist = c->scf.head = 0;
  return CF_OK;
}

cf_status chebfilter_get_H_cc(cf_ctx *c, const int32_t *cells, int64_t ncells, double *out) {
  if (!c) return CF_EINVAL;
  if (ncells < 0) return set_err(c, CF_EINVAL, "get_H_cc: bad cell count");
  if (ncells == 0) return CF_OK;
  if (!cells || !out) return set_err(c, CF_EINVAL, "get_H_cc: null argument");
  for (int64_t i = 0; i < ncells; ++i)
    if (cells[i] < 0 || cells[i] >= c->E) return set_err(c, CF_EINVAL, "get_H_cc: cell index out of range");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int npc = c->npc;
  std::vector<double> buf((size_t)NPAD * NPAD);
  for (int64_t i = 0; i < ncells; ++i) {
    HIPCHK(c, hipMemcpy(buf.data(), c->Hp + (int64_t)cells[i] * NPAD * NPAD, buf.size() * sizeof(double),
                        hipMemcpyDeviceToHost));
    for (int a = 0; a < npc; ++a)
      std::memcpy(out + (i * npc + a) * npc, buf.data() + (size_t)a * NPAD, npc * sizeof(double));
  }
  return CF_OK;
}

cf_status chebfilter_residual_norms(cf_ctx *c, const double *Z, int64_t ldz, int64_t N,
                                    const double *theta_host, double *res_host) {
  if (!c) return CF_EINVAL;
  STCHK(check_block(c, Z, ldz, N, "residual_norms Z"));
  if (N > 0 && (!theta_host || !res_host)) return set_err(c, CF_EINVAL, "residual_norms: null theta or res");
  if (N == 0) return CF_OK;
  HIPCHK(c, hipSetDevice(c->device));
  const int64_t ld = c->ldw;
  // per column chunk: T = H Z - M Z diag(theta); U = (M^E)^-1 T; res_j = sqrt(T_j . U_j)
  HIPCHK(c, hipMemcpyAsync(c->theta, theta_host, N * sizeof(double), hipMemcpyHostToDevice, c->stream));
  for (int64_t j0 = 0; j0 < N; j0 += c->chunk) {
    const int nc = (int)std::min(c->chunk, N - j0);
    STCHK(core_apply_H(c, Z + j0, ldz, c->T, ld, nc));
    STCHK(core_apply_M(c, Z + j0, ldz, c->U, ld, nc));
    HIPCHK(c, launch_sub_colscale(c->stream, c->n, nc, c->T, ld, c->U, ld, c->theta + j0));
    STCHK(core_apply_Sinv(c, c->T, ld, c->U, ld, nc));
    const int nchunks = (int)std::min<int64_t>(256, (int64_t)c->gp_chunks * c->max_cols);
    HIPCHK(c, launch_coldot(c->stream, c->n, nc, c->T, ld, c->U, ld, c->Gp, nchunks, c->evE + j0));
  }
  std::vector<double> sq(N);
  HIPCHK(c, hipMemcpyAsync(sq.data(), c->evE, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t j = 0; j < N; ++j) res_host[j] = std::sqrt(std::max(sq[j], 0.0));
  return CF_OK;
}

// Learned bounds.  history: the raw features of the last steps, oldest
// first, 8 per step: theta_1, theta_Nw, theta_N, b used, m used, largest and
// median residual norm, largest change of the wanted Ritz values.
cf_status chebfilter_bounds_features(const double *history, int32_t steps, double *out) {
  if (!history || !out || steps < 1) return CF_EINVAL;
  const double *last = history + 8 * (steps - 1);
  const double thN = last[2], w = last[3] - last[2];
  if (!(w > 0.0) || !std::isfinite(w) || !std::isfinite(thN)) return CF_EINVAL;
  for (int s = 0; s < steps; ++s) {
    const double *f = history + 8 * s;
    double *x = out + 8 * s;
    for (int q = 0; q < 4; ++q) x[q] = (f[q] - thN) / w;        // theta_1, theta_Nw, theta_N, b
    x[4] = f[4] / 100.0;                                           // degree
    for (int q = 5; q < 8; ++q) x[q] = std::log10(std::max(f[q], 0.0) / w + 1e-30);
  }
  return CF_OK;
}

// Degree rule of the learned-bounds form: the smallest m with
// T_m(|t(theta_w)|) >= rho (t(x) = (2x - a - b)/(b - a)), capped where
// T_m(|t(theta_1)|) / T_m(|t(theta_w)|) ~ exp(m (acosh|t_1| - acosh|t_w|))
// reaches 1e12 (beyond it the wanted directions near theta_w drown in the
// rounding of the lowest ones), clamped to [m_min, m_max].
cf_status chebfilter_degree_rule(double theta_1, double theta_w, double a, double b, double rho,
                                 int32_t m_min, int32_t m_max, int32_t *m) {
  if (!m || !(b > a) || !std::isfinite(a) || !std::isfinite(b) || !(rho > 1.0) || m_min < 1 ||
      m_max < m_min)
    return CF_EINVAL;
  const double t = std::fabs((2.0 * theta_w - a - b) / (b - a));
  double mr = t <= 1.0 ? INFINITY : std::ceil(std::acosh(rho) / std::acosh(t));
  const double t1 = std::fabs((2.0 * theta_1 - a - b) / (b - a));
  const double g = std::acosh(std::max(t1, 1.0)) - std::acosh(std::max(t, 1.0));
  if (g > 0.0) mr = std::min(mr, std::floor(std::log(1e12) / g));
  *m = (int32_t)std::min<double>(std::max<double>(mr, m_min), m_max);
  return CF_OK;
}

// The 8 summary numbers of one step (the network's raw inputs):
// theta_1, theta_Nw, theta_N, b used, m used, largest and median residual
// norm of the wanted pairs, largest change of the wanted Ritz values.
cf_status chebfilter_step_summary(const double *theta, const double *theta_prev, int32_t N,
                                  int32_t wanted, double b_used, int32_t m_used,
                                  const double *res, double *out) {
  if (!theta || !theta_prev || !res || !out || wanted < 1 || wanted > N) return CF_EINVAL;
  std::vector<double> r(res, res + wanted);
  double d = 0.0;
  for (int i = 0; i < wanted; ++i) d = std::max(d, std::fabs(theta[i] - theta_prev[i]));
  std::sort(r.begin(), r.end());
  const double med = (wanted % 2) ? r[wanted / 2] : 0.5 * (r[wanted / 2 - 1] + r[wanted / 2]);
  out[0] = theta[0]; out[1] = theta[wanted - 1]; out[2] = theta[N - 1];
  out[3] = b_used; out[4] = (double)m_used; out[5] = r[wanted - 1]; out[6] = med; out[7] = d;
  return CF_OK;
}

// Training sample of the learned bounds for the current operator: input =
// chebfilter_bounds_features(history); target = ((a* - theta_N)/w,
// (b* - theta_N)/w, m*) with a* = theta[N-1] (the projection of this
// operator on the current subspace), b* the upper bound of a k-step Lanczos
// run from v0, m* = chebfilter_degree_rule(theta_1, theta_Nw, a*, b*, 100,
// m_min, m_max), and theta_N, w = b - theta_N of the history's last step.
cf_status chebfilter_bounds_label(cf_ctx *c, const double *history, int32_t steps,
                                  const double *theta, int32_t N, int32_t wanted,
                                  const double *v0, int32_t k, int32_t m_min, int32_t m_max,
                                  double *input, double *target) {
  if (!c) return CF_EINVAL;
  if (!history || !theta || !v0 || !input || !target || steps < 1 || wanted < 1 || wanted > N)
    return set_err(c, CF_EINVAL, "bounds_label: bad argument");
  STCHK(chebfilter_bounds_features(history, steps, input) == CF_OK
            ? CF_OK : set_err(c, CF_EINVAL, "bounds_label: history not usable"));
  double lo = 0.0, bstar = 0.0;
  STCHK(chebfilter_lanczos_bounds(c, v0, k, &lo, &bstar));
  const double *last = history + 8 * (steps - 1);
  const double thN = last[2], w = last[3] - last[2];
  const double astar = theta[N - 1];
  int32_t mstar = 0;
  if (chebfilter_degree_rule(theta[0], theta[wanted - 1], astar, bstar, 100.0, m_min, m_max,
                             &mstar) != CF_OK)
    return set_err(c, CF_EINVAL, "bounds_label: degree rule");
  target[0] = (astar - thN) / w;
  target[1] = (bstar - thN) / w;
  target[2] = (double)mstar;
  return CF_OK;
}

cf_status chebfilter_bounds_predict(cf_ctx *c, cf_mlp *mlp, const double *history, const double *v0,
                                    int32_t lanczos_k, int32_t m_min, int32_t m_max, double *a,
                                    double *b, int32_t *m, int32_t *fallback) {
  if (!c) return CF_EINVAL;
  if (!mlp || !history || !v0 || !a || !b || !m || !fallback)
    return set_err(c, CF_EINVAL, "bounds_predict: null argument");
  if (cf_mlp_n_out(mlp) != 3 || cf_mlp_n_in(mlp) % 8 != 0)
    return set_err(c, CF_EINVAL, "bounds_predict: the network must map 8 features per step to 3 outputs");
  if (m_min < 1 || m_max < m_min) return set_err(c, CF_EINVAL, "bounds_predict: bad degree range");
  const int steps = cf_mlp_n_in(mlp) / 8;
  const double *last = history + 8 * (steps - 1);
  const double th1 = last[0], thw = last[1], thN = last[2], b_last = last[3], m_last = last[4];
  const double wlast = b_last - thN;
  bool ok = std::isfinite(th1) && std::isfinite(thw) && std::isfinite(thN) && wlast > 0.0 &&
            std::isfinite(wlast);
  double y[3] = {NAN, NAN, NAN};
  if (ok) {
    std::vector<double> x(8 * steps);
    ok = chebfilter_bounds_features(history, steps, x.data()) == CF_OK;
    if (ok) {
      cf_status st = cf_mlp_predict_raw(mlp, x.data(), y);
      if (st != CF_OK) return set_err(c, st, std::string("bounds_predict: ") + cf_mlp_err(mlp));
    }
  }
  // outputs (alpha, beta, m): a = theta_N + alpha w, b = theta_N + beta w with
  // w the last step's b - theta_N.  Guard: b must stay a safe upper bound (an
  // overestimate only costs damping; an underestimate amplifies the top of the
  // spectrum by T_m(t > 1)), so beta must lie within [0.98, 2]; a 5 % margin
  // is added
  ok = ok && std::isfinite(y[0]) && std::isfinite(y[1]) && std::isfinite(y[2]) && y[1] >= 0.98 &&
       y[1] <= 2.0;
  if (ok) {
    const double bw = y[1] * wlast;
    *b = thN + 1.05 * bw;
    const double ap = thN + y[0] * wlast;
    // a: inside [theta_Nw, theta_N + (b - theta_N)/4], else theta_N
    *a = (ap >= thw && ap <= thN + 0.25 * (*b - thN)) ? ap : thN;
    // degree: rounded, and at most the degree at which theta_1 is amplified
    // 1e12 times more than theta_Nw (beyond it the orthonormalisation cannot
    // resolve the wanted directions near theta_Nw in FP64)
    double mr = std::round(y[2]);
    const double t1 = std::fabs((2.0 * th1 - *a - *b) / (*b - *a));
    const double tw = std::fabs((2.0 * thw - *a - *b) / (*b - *a));
    const double g = std::acosh(std::max(t1, 1.0)) - std::acosh(std::max(tw, 1.0));
    if (g > 0.0) mr = std::min(mr, std::floor(std::log(1e12) / g));
    *m = (int32_t)std::min<double>(std::max<double>(mr, m_min), m_max);
    *fallback = 0;
    return CF_OK;
  }
  double lo = 0.0, bu = 0.0;
  STCHK(chebfilter_lanczos_bounds(c, v0, lanczos_k, &lo, &bu));
  *b = bu;
  *a = thN < bu ? thN : lo;
  const double mr = std::isfinite(m_last) ? std::round(m_last) : (double)m_min;
  *m = (int32_t)std::min<double>(std::max<double>(mr, m_min), m_max);
  *fallback = 1;
  return CF_OK;
}

}  // extern "C"
