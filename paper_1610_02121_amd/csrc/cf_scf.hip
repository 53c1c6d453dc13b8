// Kernels of the self-consistent field quantities around the eigensolver
// (Sec. II and Sec. V).  All fields live on the quadrature points: the plain
// cells' Gauss points, then the adaptive grid's points (Sec. IV.C).  A cell's
// points are a contiguous range of the point arrays; the basis at a point is
// evaluated from its coordinates (1D Lagrange products; the enrichment
// functions through the shared helpers).
//
//   density:  D_e = Y_e diag(2 f) Y_e^T per cell (Y_e: the block's rows of the
//             cell's nodes and enrichment functions), then
//             rho_q = Phi_q^T D_e Phi_q at every point (Eq. Rho)  -- FP64 MFMA
//   LDA:      eps_xc, V_xc per point (Perdew-Zunger fit of Ceperley-Alder)
//   Poisson:  b_j = sum_q w_q (rho - rho_g)_q N_j(x_q) (Eq. ForceCFEM), the
//             matrix A^C = K / (2 pi) per cell (Eq. discretePoissonCFEM)
//   V_H at the points by interpolation, plus the neutralising Gaussian's
//   potential; V_eff = V_ext + V_H + V_xc (Eq. veff)
//   mixing:   weighted dot products and the Anderson combination (Sec. V)
//
// MFMA fragment layout of v_mfma_f64_16x16x4f64 (wave of 64 lanes):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element r holds D[4 * r + l / 16][l % 16]
#include "cf_ea_body.h"

namespace cf {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 scf_mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// rows of the cell's block: local node r < NPAD (zero for a Dirichlet or
// padding node), then enrichment function r - NPAD < na
__device__ __forceinline__ int64_t scf_row(const ScfArgs &g, int e, int r, int na) {
  if (r < NPAD) {
    const int d = g.dofp[(int64_t)e * NPAD + r];
    return d;                                        // -1: zero row
  }
  const int s = r - NPAD;
  if (s >= na) return -1;
  return g.n_h + g.eidx[g.eptr[e] + s];
}

// ---------------------------------------------------------------------------
// D_e upper tiles of one work item (cell slot, first tile, count <= 64); the
// block's columns are walked in stages of 16 staged through LDS with the
// weights 2 f_j.
// ---------------------------------------------------------------------------
constexpr int DM_KMAX = NPAD + EA_MAXNAP;       // rows of the largest cell block
constexpr int DM_LD = 17;

__global__ __launch_bounds__(256) void k_scf_dm(const ScfArgs g, const int32_t *__restrict__ item_c,
                                                const int32_t *__restrict__ item_t0,
                                                const int32_t *__restrict__ item_nt,
                                                const double *__restrict__ X, int64_t ldx, int N,
                                                const double *__restrict__ f2,
                                                double *__restrict__ Dbuf) {
  __shared__ double Ys[DM_KMAX * DM_LD];
  __shared__ double fs[16];
  __shared__ int64_t rows[DM_KMAX];
  const int c = item_c[blockIdx.x], t0 = item_t0[blockIdx.x], ntl = item_nt[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int e = g.cell[c];
  const int na = g.cna[c];
  const int K = NPAD + ((na + 15) & ~15), nt = K / 16;
  for (int r = tid; r < K; r += 256) rows[r] = scf_row(g, e, r, na);
  d4 acc[16];
  int ti[16], tj[16];
  bool on[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    const int tl = w + 4 * u;
    on[u] = tl < ntl;
    int t = on[u] ? t0 + tl : 0, i = 0;
    while (t >= nt - i) { t -= nt - i; ++i; }
    ti[u] = i;
    tj[u] = i + t;
  }
  __syncthreads();
  for (int j0 = 0; j0 < N; j0 += 16) {
    for (int q = tid; q < K * 16; q += 256) {
      const int r = q >> 4, j = q & 15;
      const int64_t row = rows[r];
      Ys[r * DM_LD + j] = (row >= 0 && j0 + j < N) ? X[row * ldx + j0 + j] : 0.0;
    }
    if (tid < 16) fs[tid] = j0 + tid < N ? f2[j0 + tid] : 0.0;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + kq;
      const double fk = fs[k];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (!on[u]) continue;
        acc[u] = scf_mfma(Ys[(16 * ti[u] + li) * DM_LD + k] * fk, Ys[(16 * tj[u] + li) * DM_LD + k],
                          acc[u]);
      }
    }
    __syncthreads();
  }
  double *D = Dbuf + g.doff[c];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    if (!on[u]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      D[(int64_t)(16 * ti[u] + 4 * r + kq) * K + 16 * tj[u] + li] = acc[u][r];
  }
}

// ---------------------------------------------------------------------------
// Basis values at a stage of up to 16 points of a cell into LDS: Phi[q][a] for
// the NPAD local nodes (zero beyond npc) and Phi[q][NPAD + s] for the cell's
// enrichment functions (values only).
// ---------------------------------------------------------------------------
constexpr int RHO_P = 16;
constexpr int PHI_LD = DM_KMAX + 1;

__device__ void scf_stage_basis(const ScfArgs &g, const EaTab &t, int c, int64_t p0, int np,
                                int na, const int *atom, double (*L1)[3][EA_MAXNP], double *Phi,
                                int nthr) {
  const int tid = threadIdx.x, np1 = g.np1, npc = np1 * np1 * np1;
  if (tid < RHO_P * 3) {
    const int k = tid / 3, d = tid % 3;
    double dummy[EA_MAXNP];
    if (k < np) {
      const double x = g.xyz[3 * (p0 + k) + d];
      ea_lagrange(t.nodes, np1, (x - g.lo[3 * c + d]) / g.h, L1[k][d], dummy);
    } else {
      for (int i = 0; i < np1; ++i) L1[k][d][i] = 0.0;
    }
  }
  const int nat = g.npa ? na / g.npa : 0;
  if (na > 0) {
    EnrAsm ea;
    ea.centers = g.centers;
    ea.nsh = g.nsh;
    ea.r0 = g.r0;
    ea.t = g.t;
    for (int j = tid - 64; j >= 0 && j < RHO_P * nat; j += nthr - 64) {
      const int k = j / nat, u = j % nat;
      double *row = Phi + k * PHI_LD + NPAD;
      if (k < np) {
        const double x[3] = {g.xyz[3 * (p0 + k)], g.xyz[3 * (p0 + k) + 1],
                             g.xyz[3 * (p0 + k) + 2]};
        ea_atom_val(ea, t, atom[u], x, row, u * g.npa);
      } else {
        for (int m = 0; m < g.npa; ++m) row[u * g.npa + m] = 0.0;
      }
    }
  }
  __syncthreads();
  for (int q = tid; q < RHO_P * NPAD; q += nthr) {
    const int k = q / NPAD, a = q % NPAD;
    double v = 0.0;
    if (a < npc) v = L1[k][0][a % np1] * L1[k][1][(a / np1) % np1] * L1[k][2][a / (np1 * np1)];
    Phi[k * PHI_LD + a] = v;
  }
  __syncthreads();
}

// rho_q = Phi_q^T D_e Phi_q = sum over upper 16 x 16 tiles (ta <= tb) of D_e of
// (2 - [ta == tb]) (Phi_q,ta D_ta,tb) . Phi_q,tb.  One work item = (SCF cell,
// a range of at most 8 RHO_TPW upper tiles, a chunk of at most SCF_RHO_QCHUNK
// of the cell's points); its 8 waves keep their tiles of D_e in registers (as
// MFMA B fragments) for the whole chunk, so the stage loop over the points
// reads only LDS.  Items of the first tile range write rho, those of later
// ranges (cells with more tiles) add to it in a later launch; the chunks of
// one range cover distinct points.
constexpr int RHO_TPW = 12;
static_assert(8 * RHO_TPW == SCF_RHO_TILES, "density items hold 8 waves of RHO_TPW tiles");

__global__ __launch_bounds__(512) void k_scf_rho(const ScfArgs g, const int32_t *__restrict__ item_c,
                                                 const int32_t *__restrict__ item_t0,
                                                 const int32_t *__restrict__ item_nt,
                                                 const int32_t *__restrict__ item_q0, int add,
                                                 const double *__restrict__ Dbuf,
                                                 double *__restrict__ rho) {
  __shared__ double stab[EA_TAB_MAX];
  __shared__ double L1[RHO_P][3][EA_MAXNP];
  __shared__ double Phi[RHO_P * PHI_LD];
  __shared__ double part[8][RHO_P];
  __shared__ int atom[EA_MAXNAP];
  const int c = item_c[blockIdx.x], t0 = item_t0[blockIdx.x], ntl = item_nt[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  for (int i = tid; i < g.ntab; i += 512) stab[i] = g.tab[i];
  const int e = g.cell[c];
  const int na = g.cna[c];
  if (na > 0)
    for (int u = tid; u < na / g.npa; u += 512) atom[u] = g.eidx[g.eptr[e] + (int64_t)u * g.npa] / g.npa;
  for (int i = tid; i < RHO_P * PHI_LD; i += 512) Phi[i] = 0.0;
  const int K = NPAD + ((na + 15) & ~15), nt = K / 16;
  const double *D = Dbuf + g.doff[c];
  // this wave's tiles and their D fragments: B[k][j] = D[16 ta + k][16 tb + j]
  int ta[RHO_TPW], tb[RHO_TPW];
  bool on[RHO_TPW];
  double dB[RHO_TPW][4];
#pragma unroll
  for (int u = 0; u < RHO_TPW; ++u) {
    const int tl = w + 8 * u;
    on[u] = tl < ntl;
    int t = on[u] ? t0 + tl : 0, i = 0;
    while (t >= nt - i) { t -= nt - i; ++i; }
    ta[u] = i;
    tb[u] = i + t;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      dB[u][s] = on[u] ? D[(int64_t)(16 * ta[u] + 4 * s + kq) * K + 16 * tb[u] + li] : 0.0;
  }
  __syncthreads();
  EaTab t;
  {
    EnrAsm ea;
    ea.np1 = g.np1;
    ea.ng = g.ng;
    ea.nsh = g.nsh;
    t = ea_tab(stab, ea);
  }
  // this item's chunk of the cell's points
  const int64_t p0 = g.pofs[c] + item_q0[blockIdx.x];
  const int64_t np = min<int64_t>(SCF_RHO_QCHUNK, g.pcnt[c] - item_q0[blockIdx.x]);
  for (int64_t q0 = 0; q0 < np; q0 += RHO_P) {
    const int ns = (int)min<int64_t>(RHO_P, np - q0);
    scf_stage_basis(g, t, c, p0 + q0, ns, na, atom, L1, Phi, 512);
    double pr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < RHO_TPW; ++u) {
      if (!on[u]) continue;
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        acc = scf_mfma(Phi[li * PHI_LD + 16 * ta[u] + 4 * s + kq], dB[u][s], acc);
      const double f = ta[u] == tb[u] ? 1.0 : 2.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) pr[r] += f * acc[r] * Phi[(4 * r + kq) * PHI_LD + 16 * tb[u] + li];
    }
    // sum over the 16 lanes of a row group (li), then over the waves in order
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = pr[r];
      for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 16);
      pr[r] = v;
    }
    if (li == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) part[w][4 * r + kq] = pr[r];
    }
    __syncthreads();
    if (tid < ns) {
      double v = part[0][tid];
      for (int k = 1; k < 8; ++k) v += part[k][tid];
      rho[p0 + q0 + tid] = add ? rho[p0 + q0 + tid] + v : v;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LDA (Perdew-Zunger fit of the Ceperley-Alder correlation, Slater exchange),
// and per-block partial sums of w rho, w rho eps_xc, w rho V_xc.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scf_lda(double rho, double &eps, double &v) {
  if (!(rho > 1e-30)) { eps = 0.0; v = 0.0; return; }
  constexpr double PI = 3.14159265358979323846;
  const double cr = cbrt(rho);
  const double ex = -0.75 * cbrt(3.0 / PI) * cr;
  const double rs = cbrt(3.0 / (4.0 * PI * rho));
  double ec, vc;
  if (rs >= 1.0) {
    const double s = sqrt(rs);
    const double den = 1.0 + 1.0529 * s + 0.3334 * rs;
    ec = -0.1423 / den;
    const double dec = 0.1423 * (0.5 * 1.0529 / s + 0.3334) / (den * den);
    vc = ec - rs / 3.0 * dec;
  } else {
    const double lr = log(rs);
    ec = 0.0311 * lr - 0.048 + 0.0020 * rs * lr - 0.0116 * rs;
    const double dec = 0.0311 / rs + 0.0020 * (lr + 1.0) - 0.0116;
    vc = ec - rs / 3.0 * dec;
  }
  eps = ex + ec;
  v = 4.0 / 3.0 * ex + vc;
}

__global__ __launch_bounds__(256) void k_scf_lda(int64_t P, const double *__restrict__ rho,
                                                 const double *__restrict__ w,
                                                 double *__restrict__ vxc,
                                                 double *__restrict__ partials) {
  __shared__ double red[3][256];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
    double eps, v;
    scf_lda(rho[p], eps, v);
    vxc[p] = v;
    const double wr = w[p] * rho[p];
    s0 += wr;
    s1 += wr * eps;
    s2 += wr * v;
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 3) partials[(int64_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// the neutralising Gaussian at a point: density and potential
__device__ __forceinline__ void scf_gauss(const ScfArgs &g, const double *x, double &rg,
                                          double &vg) {
  constexpr double PI = 3.14159265358979323846;
  const double dx = x[0] - g.cc[0], dy = x[1] - g.cc[1], dz = x[2] - g.cc[2];
  const double d = sqrt(dx * dx + dy * dy + dz * dz);
  const double s = g.cs;
  rg = g.Q / (s * s * s * PI * sqrt(PI)) * exp(-(d / s) * (d / s));
  vg = d < 1e-8 * s ? g.Q * 2.0 / (sqrt(PI) * s) : g.Q * erf(d / s) / d;
}

// the neutralising Gaussian's density at a point
__device__ __forceinline__ double scf_gauss_rho(const ScfArgs &g, const double *x) {
  constexpr double PI = 3.14159265358979323846;
  const double dx = x[0] - g.cc[0], dy = x[1] - g.cc[1], dz = x[2] - g.cc[2];
  const double s = g.cs;
  return g.Q / (s * s * s * PI * sqrt(PI)) * exp(-(dx * dx + dy * dy + dz * dz) / (s * s));
}

// ---------------------------------------------------------------------------
// Poisson right-hand side of the cells of one colour: b[dof(e,a)] += sum_q
// w_q (rho - rho_g)_q N_a(x_q).  128 threads; a stage is 128 points, thread k
// evaluating point k's 1D Lagrange values and weight, then thread a summing
// over the stage's points for its node a.
// ---------------------------------------------------------------------------
constexpr int RHS_P = NPAD;

__global__ __launch_bounds__(NPAD) void k_scf_rhs(const ScfArgs g, const int32_t *__restrict__ cells,
                                                  const double *__restrict__ rho,
                                                  double *__restrict__ b) {
  __shared__ double stab[EA_TAB_MAX];
  __shared__ double L1[RHS_P][3][EA_MAXNP];
  __shared__ double sv[RHS_P];
  const int c = cells[blockIdx.x];
  const int tid = threadIdx.x, np1 = g.np1, npc = np1 * np1 * np1;
  for (int i = tid; i < g.ntab; i += NPAD) stab[i] = g.tab[i];
  __syncthreads();
  const double *nodes = stab;
  const int e = g.cell[c];
  const int64_t p0 = g.pofs[c], np = g.pcnt[c];
  const int i0 = tid % np1, i1 = (tid / np1) % np1, i2 = tid / (np1 * np1);
  double acc = 0.0;
  for (int64_t q0 = 0; q0 < np; q0 += RHS_P) {
    const int ns = (int)min<int64_t>(RHS_P, np - q0);
    if (tid < ns) {
      const int64_t p = p0 + q0 + tid;
      double dummy[EA_MAXNP];
      for (int d = 0; d < 3; ++d)
        ea_lagrange(nodes, np1, (g.xyz[3 * p + d] - g.lo[3 * c + d]) / g.h, L1[tid][d], dummy);
      sv[tid] = g.w[p] * (rho[p] - scf_gauss_rho(g, g.xyz + 3 * p));
    }
    __syncthreads();
    if (tid < npc)
      for (int k = 0; k < ns; ++k) acc += sv[k] * (L1[k][0][i0] * L1[k][1][i1] * L1[k][2][i2]);
    __syncthreads();
  }
  if (tid < npc) {
    const int d = g.dofp[(int64_t)e * NPAD + tid];
    if (d >= 0) b[d] += acc;
  }
}

// y[dof(e,a)] += sum_b A[a][b] x[dof(e,b)] for the cells of one colour, one
// matrix for every cell (the uniform mesh's A^C block); thread a.
__global__ __launch_bounds__(NPAD) void k_scf_lap(const ScfArgs g, const int32_t *__restrict__ cells,
                                                  const double *__restrict__ A,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ y) {
  __shared__ double xs[NPAD];
  const int e = g.cell[cells[blockIdx.x]];
  const int a = threadIdx.x;
  const int d = g.dofp[(int64_t)e * NPAD + a];
  xs[a] = d >= 0 ? x[d] : 0.0;
  __syncthreads();
  if (d < 0) return;
  double s = 0.0;
  for (int k = 0; k < NPAD; ++k) s = fma(A[k * NPAD + a], xs[k], s);
  y[d] += s;
}

// CG helpers on n-vectors: op 0: z = dinv .* r; op 1: p = z + beta p;
// op 2: x += alpha p, r -= alpha q; op 3: r = z - q (z holding b)
__global__ __launch_bounds__(256) void k_scf_cg(int64_t n, int op, double alpha, double beta,
                                                const double *__restrict__ dinv,
                                                double *__restrict__ x, double *__restrict__ r,
                                                double *__restrict__ z, double *__restrict__ p,
                                                const double *__restrict__ q) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (op == 0) {
      z[i] = dinv[i] * r[i];
    } else if (op == 1) {
      p[i] = z[i] + beta * p[i];
    } else if (op == 2) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    } else {
      r[i] = z[i] - q[i];
    }
  }
}

// CG steps with the scalars on the device (sc: 0 r.z, 1 p.q, 2 r.r, 3 new r.z,
// 4 alpha, 5 beta): op 0: alpha = r.z / p.q; op 1: x += alpha p, r -= alpha q,
// z = dinv .* r; op 2: beta = new r.z / r.z, r.z = new r.z; op 3: p = z + beta p
__global__ __launch_bounds__(256) void k_scf_cgd(int64_t n, int op, double *__restrict__ sc,
                                                 const double *__restrict__ dinv,
                                                 double *__restrict__ x, double *__restrict__ r,
                                                 double *__restrict__ z, double *__restrict__ p,
                                                 const double *__restrict__ q) {
  if (op == 0 || op == 2) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (op == 0) {
        sc[4] = sc[0] / sc[1];
      } else {
        sc[5] = sc[3] / sc[0];
        sc[0] = sc[3];
      }
    }
    return;
  }
  const double alpha = sc[4], beta = sc[5];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (op == 1) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      z[i] = dinv[i] * ri;
    } else {
      p[i] = z[i] + beta * p[i];
    }
  }
}

// V_H at the points of one cell per workgroup (interpolation of Phi plus the
// Gaussian's potential), V_eff = V_ext + V_H + V_xc, and the block partial
// sum of w rho V_H.
__global__ __launch_bounds__(256) void k_scf_veff(const ScfArgs g, const double *__restrict__ phi,
                                                  const double *__restrict__ rho,
                                                  const double *__restrict__ vext,
                                                  const double *__restrict__ vxc,
                                                  double *__restrict__ veff,
                                                  double *__restrict__ partials) {
  __shared__ double stab[EA_TAB_MAX];
  __shared__ double ph[NPAD];
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, np1 = g.np1, npc = np1 * np1 * np1;
  for (int i = tid; i < g.ntab; i += 256) stab[i] = g.tab[i];
  const int e = g.cell[c];
  if (tid < NPAD) {
    const int d = g.dofp[(int64_t)e * NPAD + tid];
    ph[tid] = (d >= 0 && tid < npc) ? phi[d] : 0.0;
  }
  __syncthreads();
  const int64_t p0 = g.pofs[c], np = g.pcnt[c];
  double s = 0.0;
  for (int64_t q = tid; q < np; q += 256) {
    const int64_t p = p0 + q;
    double L[3][EA_MAXNP], dummy[EA_MAXNP];
    for (int d = 0; d < 3; ++d) ea_lagrange(stab, np1, (g.xyz[3 * p + d] - g.lo[3 * c + d]) / g.h, L[d], dummy);
    double v = 0.0;
    for (int k2 = 0; k2 < np1; ++k2)
      for (int k1 = 0; k1 < np1; ++k1) {
        const double lyz = L[1][k1] * L[2][k2];
        const double *prow = ph + (k2 * np1 + k1) * np1;
        double t = 0.0;
        for (int k0 = 0; k0 < np1; ++k0) t += L[0][k0] * prow[k0];
        v += lyz * t;
      }
    double rg, vg;
    scf_gauss(g, g.xyz + 3 * p, rg, vg);
    const double vh = v + vg;
    veff[p] = vext[p] + vh + vxc[p];
    s += g.w[p] * rho[p] * vh;
  }
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) partials[c] = red[0];
}

// partial sums of w a b over blocks of points (fixed grid; summed in order on the host)
__global__ __launch_bounds__(256) void k_scf_wdot(int64_t P, const double *__restrict__ w,
                                                  const double *__restrict__ a,
                                                  const double *__restrict__ b,
                                                  double *__restrict__ partials) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256)
    s += w[p] * a[p] * b[p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// out = sum_k c_k (rin_k + beta F_k) over the history slots (k < m <= 8)
__global__ __launch_bounds__(256) void k_scf_mix(int64_t P, int m, ScfMixCoef cf, double beta,
                                                 const double *__restrict__ rin,
                                                 const double *__restrict__ F, int64_t ld,
                                                 double *__restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += cf.c[k] * (rin[k * ld + p] + beta * F[k * ld + p]);
    out[p] = v;
  }
}

// F = rho_out - rho_in into history slot k (and rho_in into its slot)
__global__ __launch_bounds__(256) void k_scf_push(int64_t P, const double *__restrict__ rin,
                                                  const double *__restrict__ rout,
                                                  double *__restrict__ hin, double *__restrict__ hF) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
    hin[p] = rin[p];
    hF[p] = rout[p] - rin[p];
  }
}

// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

hipError_t launch_scf_dm(hipStream_t s, const ScfArgs &g, int nitems, const int32_t *item_c,
                         const int32_t *item_t0, const int32_t *item_nt, const double *X,
                         int64_t ldx, int N, const double *f2, double *Dbuf) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scf_dm, dim3((unsigned)nitems), dim3(256), 0, s, g, item_c, item_t0,
                     item_nt, X, ldx, N, f2, Dbuf);
  return hipGetLastError();
}

hipError_t launch_scf_rho(hipStream_t s, const ScfArgs &g, int nitems, const int32_t *item_c,
                          const int32_t *item_t0, const int32_t *item_nt, const int32_t *item_q0,
                          int add, const double *Dbuf, double *rho) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scf_rho, dim3((unsigned)nitems), dim3(512), 0, s, g, item_c, item_t0,
                     item_nt, item_q0, add, Dbuf, rho);
  return hipGetLastError();
}

hipError_t launch_scf_lda(hipStream_t s, int64_t P, const double *rho, const double *w, double *vxc,
                          double *partials, int nblocks) {
  hipLaunchKernelGGL(k_scf_lda, dim3((unsigned)nblocks), dim3(256), 0, s, P, rho, w, vxc, partials);
  return hipGetLastError();
}

hipError_t launch_scf_rhs(hipStream_t s, const ScfArgs &g, int ncells, const int32_t *cells,
                          const double *rho, double *b) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scf_rhs, dim3((unsigned)ncells), dim3(NPAD), 0, s, g, cells, rho, b);
  return hipGetLastError();
}

hipError_t launch_scf_lap(hipStream_t s, const ScfArgs &g, int ncells, const int32_t *cells,
                          const double *A, const double *x, double *y) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scf_lap, dim3((unsigned)ncells), dim3(NPAD), 0, s, g, cells, A, x, y);
  return hipGetLastError();
}

hipError_t launch_scf_cg(hipStream_t s, int64_t n, int op, double alpha, double beta,
                         const double *dinv, double *x, double *r, double *z, double *p,
                         const double *q) {
  hipLaunchKernelGGL(k_scf_cg, dim3(grid_for(n)), dim3(256), 0, s, n, op, alpha, beta, dinv, x, r, z,
                     p, q);
  return hipGetLastError();
}

hipError_t launch_scf_cgd(hipStream_t s, int64_t n, int op, double *sc, const double *dinv,
                          double *x, double *r, double *z, double *p, const double *q) {
  const unsigned grid = (op == 0 || op == 2) ? 1u : grid_for(n);
  hipLaunchKernelGGL(k_scf_cgd, dim3(grid), dim3(256), 0, s, n, op, sc, dinv, x, r, z, p, q);
  return hipGetLastError();
}

hipError_t launch_scf_veff(hipStream_t s, const ScfArgs &g, int ncells, const double *phi,
                           const double *rho, const double *vext, const double *vxc, double *veff,
                           double *partials) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scf_veff, dim3((unsigned)ncells), dim3(256), 0, s, g, phi, rho, vext, vxc,
                     veff, partials);
  return hipGetLastError();
}

hipError_t launch_scf_wdot(hipStream_t s, int64_t P, const double *w, const double *a,
                           const double *b, double *partials, int nblocks) {
  hipLaunchKernelGGL(k_scf_wdot, dim3((unsigned)nblocks), dim3(256), 0, s, P, w, a, b, partials);
  return hipGetLastError();
}

hipError_t launch_scf_mix(hipStream_t s, int64_t P, int m, const ScfMixCoef &cf, double beta,
                          const double *rin, const double *F, int64_t ld, double *out) {
  hipLaunchKernelGGL(k_scf_mix, dim3(grid_for(P)), dim3(256), 0, s, P, m, cf, beta, rin, F, ld, out);
  return hipGetLastError();
}

hipError_t launch_scf_push(hipStream_t s, int64_t P, const double *rin, const double *rout,
                           double *hin, double *hF) {
  hipLaunchKernelGGL(k_scf_push, dim3(grid_for(P)), dim3(256), 0, s, P, rin, rout, hin, hF);
  return hipGetLastError();
}

}  // namespace cf
