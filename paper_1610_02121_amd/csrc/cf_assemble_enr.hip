// Element blocks of the cells that carry their own adaptive quadrature rule
// (Sec. IV.C): the cells inside enrichment supports, and any plain cell given
// such a rule (e.g. one touching a bare nucleus).  The rule of a cell is a list
// of boxes (the leaves of the divide-and-conquer refinement), each carrying the
// same ng^3 Gauss rule.  With w_q the weights (box volume times the Gauss
// weights) and V_q the potential at the points (Eq. HBlocks):
//
//   H^cc_e[a,b]   = K[a,b] + sum_q w_q V_q N_a N_b                       (k_ea_nn)
//   H^ec_e[al,a]  = sum_q (w_q V_q N_al N_a + w_q/2 grad N_al . grad N_a)  (k_ea_erow)
//   H^ee_e[al,be] = sum_q (w_q V_q N_al N_be + w_q/2 grad N_al . grad N_be)
//
// N_a is the tensor-product Lagrange basis through the 1D nodes (x fastest), N_al
// an enrichment function: radial part (a sum of Slater-type terms
// c r^k exp(-zeta r)) times a real harmonic (l = 0, or l = 1 in the order
// y, z, x), times the smooth cutoff h of Eq. Moll1 (Sec. IV.B).  Every sum over
// points is a dense contraction: FP64 MFMA with the points as the k dimension,
// four points per step.  Basis values of a stage of points are evaluated by
// the workgroup into LDS first.  H^ee_e goes to a per-cell partial buffer; a
// separate kernel sums the partials of the cells in a fixed order (no atomics).
//
// MFMA fragment layout of v_mfma_f64_16x16x4f64 (wave of 64 lanes):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element r holds D[4 * r + l / 16][l % 16]
#include "cf_ea_body.h"

namespace cf {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 ea_mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// H^cc_e of every listed cell: one workgroup (4 waves) per slot; the 36 tiles
// (ti <= tj) of the upper triangle of the padded 128 x 128 block, 9 per wave.
// Stages of 16 points: the 1D Lagrange values (3 axes) and w_q V_q per point,
// then N_a at every (point, a) into LDS, then 4 MFMA steps per tile.
// ---------------------------------------------------------------------------
constexpr int NN_P = 16;

__device__ __forceinline__ int up_row(int t) {
  int i = 0;
  while (t >= 8 - i) { t -= 8 - i; ++i; }
  return i;
}
__device__ __forceinline__ int up_col(int t) {
  int i = 0;
  while (t >= 8 - i) { t -= 8 - i; ++i; }
  return i + t;
}

// the 36 upper tiles of H^cc_e into the cell's padded block (K + value at
// (row <= col), mirrored)
__device__ __forceinline__ void ea_nn_store(const EnrAsm &a, int slot, const int *ti, const int *tj,
                                            const d4 *acc) {
  const int lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
  double *He = a.Hp + (int64_t)a.cell[slot] * NPAD * NPAD;
#pragma unroll
  for (int u = 0; u < 9; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = 4 * r + kq;
      if (ti[u] == tj[u] && lr > li) continue;
      const int row = 16 * ti[u] + lr, col = 16 * tj[u] + li;
      const double v = a.K[row * NPAD + col] + acc[u][r];
      He[row * NPAD + col] = v;
      if (row != col) He[col * NPAD + row] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_ea_nn(const EnrAsm a) {
  __shared__ double stab[EA_TAB_MAX];
  __shared__ double L1[NN_P][3][EA_MAXNP];
  __shared__ double sV[NN_P];
  __shared__ double Nv[NN_P][NPAD];
  const int slot = a.nn_slot[blockIdx.x];
  const int64_t qb = a.nn_q0[blockIdx.x], qe = qb + a.nn_qn[blockIdx.x];
  const int pi = a.nn_pi[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int ntab = ea_tab_size(a.np1, a.ng, a.nsh, a.nterm);
  for (int i = tid; i < ntab; i += 256) stab[i] = a.tab[i];
  __syncthreads();
  const EaTab t = ea_tab(stab, a);
  const int np1 = a.np1, npc = np1 * np1 * np1;
  const double lo[3] = {a.lo[3 * slot], a.lo[3 * slot + 1], a.lo[3 * slot + 2]};
  d4 acc[9];
#pragma unroll
  for (int u = 0; u < 9; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
  int ti[9], tj[9];
#pragma unroll
  for (int u = 0; u < 9; ++u) { ti[u] = up_row(w + 4 * u); tj[u] = up_col(w + 4 * u); }
  for (int64_t q0 = qb; q0 < qe; q0 += NN_P) {
    if (tid < NN_P * 3) {
      const int k = tid / 3, d = tid % 3;
      double x[3], wt, v;
      double dummy[EA_MAXNP];
      if (q0 + k < qe && ea_point(a, t, slot, q0 + k, x, wt, v)) {
        ea_lagrange(t.nodes, np1, (x[d] - lo[d]) / a.h, L1[k][d], dummy);
        if (d == 0) sV[k] = wt * v;
      } else {
        for (int i = 0; i < np1; ++i) L1[k][d][i] = 0.0;
        if (d == 0) sV[k] = 0.0;
      }
    }
    __syncthreads();
    for (int e = tid; e < NN_P * NPAD; e += 256) {
      const int k = e / NPAD, c = e % NPAD;
      double v = 0.0;
      if (c < npc) v = L1[k][0][c % np1] * L1[k][1][(c / np1) % np1] * L1[k][2][c / (np1 * np1)];
      Nv[k][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < NN_P / 4; ++ks) {
      const int k = 4 * ks + kq;
      const double s = sV[k];
#pragma unroll
      for (int u = 0; u < 9; ++u)
        acc[u] = ea_mfma(Nv[k][16 * ti[u] + li] * s, Nv[k][16 * tj[u] + li], acc[u]);
    }
    __syncthreads();
  }
  if (pi < 0) {
    ea_nn_store(a, slot, ti, tj, acc);
    return;
  }
  double *P = a.Pnn + (int64_t)pi * 36 * 256;
#pragma unroll
  for (int u = 0; u < 9; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) P[(w + 4 * u) * 256 + r * 64 + lane] = acc[u][r];
}

// the partial H^cc tiles of a split slot, summed in chunk order
__global__ __launch_bounds__(256) void k_ea_nn_fin(const EnrAsm a) {
  const int slot = a.nnf_slot[blockIdx.x], p0 = a.nnf_p0[blockIdx.x], np = a.nnf_np[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  d4 acc[9];
  int ti[9], tj[9];
#pragma unroll
  for (int u = 0; u < 9; ++u) {
    ti[u] = up_row(w + 4 * u);
    tj[u] = up_col(w + 4 * u);
    acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < np; ++k) {
      const double *P = a.Pnn + (int64_t)(p0 + k) * 36 * 256 + (w + 4 * u) * 256 + lane;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[u][r] += P[r * 64];
    }
  }
  ea_nn_store(a, slot, ti, tj, acc);
}

// ---------------------------------------------------------------------------
// Enrichment rows: work item = (slot, first tile, tile count <= 4 EA_TPW).  The
// slot's tiles are the enriched-classical tiles (ti, tj), ti < nap/16, tj < 8,
// row by row, then the upper enriched-enriched tiles (ti <= tj) row by row.
// Wave w takes the item's tiles w, w + 4, ...  Each stage is EA_P points (two
// MFMA steps): the 1D Lagrange values and derivatives, the weights, then every
// enrichment function's value and gradient (one thread per (point, atom)), then
// N_a and its gradient; per tile and step 4 MFMAs (the potential term and the
// three gradient terms) with A = scaled enrichment values, B = the column
// functions.
// ---------------------------------------------------------------------------
constexpr int EA_P = 8;                        // points per stage of the enrichment rows

__device__ __forceinline__ void ea_tile(int t, int nte, int &ti, int &tj, bool &ee) {
  if (t < 8 * nte) { ti = t / 8; tj = t % 8; ee = false; return; }
  int u = t - 8 * nte, i = 0;
  while (u >= nte - i) { u -= nte - i; ++i; }
  ti = i; tj = i + u; ee = true;
}

// the tiles of an enrichment-row item into H^ec (both layouts) or the slot's
// partial H^ee block
__device__ __forceinline__ void ea_erow_store(const EnrAsm &a, int slot, const int *ti,
                                              const int *tj, const bool *ee, const bool *on,
                                              const d4 *acc) {
  const int lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
  const int e = a.cell[slot];
  const int64_t e0 = a.eptr[e];
  const int na = (int)(a.eptr[e + 1] - e0), nap = a.tld[e];
  double *Pe = a.Pee ? a.Pee + a.pee_off[slot] : nullptr;
#pragma unroll
  for (int u = 0; u < EA_TPW; ++u) {
    if (!on[u]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int al = 16 * ti[u] + 4 * r + kq;
      const int col = 16 * tj[u] + li;
      if (ee[u]) {
        Pe[(int64_t)al * nap + col] = acc[u][r];
      } else if (al < na) {
        a.Hec[(e0 + al) * NPAD + col] = acc[u][r];
        a.HT[a.toff[e] + (int64_t)col * nap + al] = acc[u][r];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_ea_erow(const EnrAsm a) {
  __shared__ double stab[EA_TAB_MAX];
  __shared__ double L1[EA_P][3][2][EA_MAXNP];
  __shared__ double sV[EA_P], sK[EA_P];
  __shared__ double Nv[4][EA_P][NPAD];         // [channel][point][a]
  __shared__ double Ev[4][EA_P][EA_MAXNAP];    // [channel][point][alpha]
  __shared__ int atom[EA_MAXNAP];
  const int item = blockIdx.x;
  const int slot = a.item_slot[item], t0 = a.item_t0[item], ntl = a.item_nt[item];
  const int64_t qb = a.item_q0[item], qe = qb + a.item_qn[item];
  const int pi = a.item_pi[item];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int ntab = ea_tab_size(a.np1, a.ng, a.nsh, a.nterm);
  for (int i = tid; i < ntab; i += 256) stab[i] = a.tab[i];
  const int e = a.cell[slot];
  const int64_t e0 = a.eptr[e];
  const int na = (int)(a.eptr[e + 1] - e0), nap = a.tld[e], nte = nap / 16;
  const int nat = na / a.npa;
  for (int u = tid; u < nat; u += 256) atom[u] = a.eidx[e0 + (int64_t)u * a.npa] / a.npa;
  // padding columns of the enrichment rows stay zero for the whole call
  for (int i = tid; i < 4 * EA_P * EA_MAXNAP; i += 256) (&Ev[0][0][0])[i] = 0.0;
  __syncthreads();
  const EaTab t = ea_tab(stab, a);
  const int np1 = a.np1, npc = np1 * np1 * np1;
  const double lo[3] = {a.lo[3 * slot], a.lo[3 * slot + 1], a.lo[3 * slot + 2]};

  d4 acc[EA_TPW];
  int ti[EA_TPW], tj[EA_TPW];
  bool ee[EA_TPW], on[EA_TPW];
#pragma unroll
  for (int u = 0; u < EA_TPW; ++u) {
    acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    const int tl = w + 4 * u;
    on[u] = tl < ntl;
    ea_tile(on[u] ? t0 + tl : 0, nte, ti[u], tj[u], ee[u]);
  }
  for (int64_t q0 = qb; q0 < qe; q0 += EA_P) {
    if (tid < 3 * EA_P) {
      const int k = tid / 3, d = tid % 3;
      double x[3], wt, v;
      if (q0 + k < qe && ea_point(a, t, slot, q0 + k, x, wt, v)) {
        ea_lagrange(t.nodes, np1, (x[d] - lo[d]) / a.h, L1[k][d][0], L1[k][d][1]);
        for (int i = 0; i < np1; ++i) L1[k][d][1][i] /= a.h;
        if (d == 0) { sV[k] = wt * v; sK[k] = 0.5 * wt; }
      } else {
        for (int i = 0; i < np1; ++i) { L1[k][d][0][i] = 0.0; L1[k][d][1][i] = 0.0; }
        if (d == 0) { sV[k] = 0.0; sK[k] = 0.0; }
      }
    }
    for (int j = tid - 64; j >= 0 && j < EA_P * nat; j += 192) {
      const int k = j / nat, u = j % nat;
      double x[3], wt, v;
      if (q0 + k < qe && ea_point(a, t, slot, q0 + k, x, wt, v)) {
        ea_atom(a, t, atom[u], x, Ev[0][k], Ev[1][k], Ev[2][k], Ev[3][k], u * a.npa);
      } else {
        for (int m = 0; m < a.npa; ++m) {
          Ev[0][k][u * a.npa + m] = 0.0; Ev[1][k][u * a.npa + m] = 0.0;
          Ev[2][k][u * a.npa + m] = 0.0; Ev[3][k][u * a.npa + m] = 0.0;
        }
      }
    }
    __syncthreads();
    for (int j = tid; j < EA_P * NPAD; j += 256) {
      const int k = j / NPAD, c = j % NPAD;
      double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
      if (c < npc) {
        const int i0 = c % np1, i1 = (c / np1) % np1, i2 = c / (np1 * np1);
        const double lx = L1[k][0][0][i0], ly = L1[k][1][0][i1], lz = L1[k][2][0][i2];
        v0 = lx * ly * lz;
        v1 = L1[k][0][1][i0] * ly * lz;
        v2 = lx * L1[k][1][1][i1] * lz;
        v3 = lx * ly * L1[k][2][1][i2];
      }
      Nv[0][k][c] = v0; Nv[1][k][c] = v1; Nv[2][k][c] = v2; Nv[3][k][c] = v3;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < EA_P / 4; ++ks) {
      const int k = 4 * ks + kq;
      const double s0 = sV[k], s1 = sK[k];
#pragma unroll
      for (int u = 0; u < EA_TPW; ++u) {
        if (!on[u]) continue;
        const int ra = 16 * ti[u] + li;
        const double a0 = Ev[0][k][ra] * s0, a1 = Ev[1][k][ra] * s1, a2 = Ev[2][k][ra] * s1,
                     a3 = Ev[3][k][ra] * s1;
        const int cb = 16 * tj[u] + li;
        double b0, b1, b2, b3;
        if (ee[u]) {
          b0 = Ev[0][k][cb]; b1 = Ev[1][k][cb]; b2 = Ev[2][k][cb]; b3 = Ev[3][k][cb];
        } else {
          b0 = Nv[0][k][cb]; b1 = Nv[1][k][cb]; b2 = Nv[2][k][cb]; b3 = Nv[3][k][cb];
        }
        acc[u] = ea_mfma(a0, b0, acc[u]);
        acc[u] = ea_mfma(a1, b1, acc[u]);
        acc[u] = ea_mfma(a2, b2, acc[u]);
        acc[u] = ea_mfma(a3, b3, acc[u]);
      }
    }
    __syncthreads();
  }
  if (pi < 0) {
    ea_erow_store(a, slot, ti, tj, ee, on, acc);
    return;
  }
  double *P = a.Ptile + (int64_t)pi * 4 * EA_TPW * 256;
#pragma unroll
  for (int u = 0; u < EA_TPW; ++u) {
    if (!on[u]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) P[(w + 4 * u) * 256 + r * 64 + lane] = acc[u][r];
  }
}

// the partial tiles of a split slot's item group, summed in chunk order
__global__ __launch_bounds__(256) void k_ea_erow_fin(const EnrAsm a) {
  const int g = blockIdx.x;
  const int slot = a.fin_slot[g], t0 = a.fin_t0[g], ntl = a.fin_nt[g];
  const int p0 = a.fin_p0[g], np = a.fin_np[g];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = a.cell[slot];
  const int nte = a.tld[e] / 16;
  d4 acc[EA_TPW];
  int ti[EA_TPW], tj[EA_TPW];
  bool ee[EA_TPW], on[EA_TPW];
#pragma unroll
  for (int u = 0; u < EA_TPW; ++u) {
    const int tl = w + 4 * u;
    on[u] = tl < ntl;
    ea_tile(on[u] ? t0 + tl : 0, nte, ti[u], tj[u], ee[u]);
    acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    if (!on[u]) continue;
    for (int k = 0; k < np; ++k) {
      const double *P = a.Ptile + (int64_t)(p0 + k) * 4 * EA_TPW * 256 + tl * 256 + lane;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[u][r] += P[r * 64];
    }
  }
  ea_erow_store(a, slot, ti, tj, ee, on, acc);
}

// ---------------------------------------------------------------------------
// H^ee from the per-cell partials: one workgroup per atom pair (I <= J) with
// the list of its cells (slot, position of I, position of J in the cell's atom
// list), in slot order.  Thread (m1, m2) sums the partial entries of its
// function pair over the list (upper-triangle entry of each partial, the
// partials being stored for alpha <= beta) and adds the sum to H^ee[al][be]
// and H^ee[be][al].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ea_ee_reduce(const EnrAsm a, int n_e,
                                                      const int32_t *__restrict__ pair_ij,
                                                      const int64_t *__restrict__ pair_ptr,
                                                      const int32_t *__restrict__ pc,
                                                      double *__restrict__ Hee) {
  const int p = blockIdx.x;
  const int I = pair_ij[2 * p], J = pair_ij[2 * p + 1];
  const int npa = a.npa;
  for (int idx = threadIdx.x; idx < npa * npa; idx += 256) {
    const int m1 = idx / npa, m2 = idx % npa;
    if (I == J && m1 > m2) continue;
    double s = 0.0;
    for (int64_t q = pair_ptr[p]; q < pair_ptr[p + 1]; ++q) {
      const int slot = pc[3 * q], ui = pc[3 * q + 1], uj = pc[3 * q + 2];
      const int nap = a.tld[a.cell[slot]];
      int l1 = ui * npa + m1, l2 = uj * npa + m2;
      if (l1 > l2) { const int tmp = l1; l1 = l2; l2 = tmp; }
      s += a.Pee[a.pee_off[slot] + (int64_t)l1 * nap + l2];
    }
    const int64_t al = (int64_t)I * npa + m1, be = (int64_t)J * npa + m2;
    const double v = Hee[al * n_e + be] + s;
    Hee[al * n_e + be] = v;
    if (al != be) Hee[be * n_e + al] = v;
  }
}

// X[i][j] = (i == j0 + j) for i < rows, j < N (unit columns j0 .. j0 + N - 1)
__global__ __launch_bounds__(256) void k_unit_cols(int64_t rows, int N, int64_t ldx, int64_t j0,
                                                   double *__restrict__ X) {
  const int64_t total = rows * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / N;
    const int j = (int)(e - i * N);
    X[i * ldx + j] = (i == j0 + j) ? 1.0 : 0.0;
  }
}

hipError_t launch_ea_nn(hipStream_t s, const EnrAsm &a, int nitems, int nfin) {
  if (nitems > 0) hipLaunchKernelGGL(k_ea_nn, dim3((unsigned)nitems), dim3(256), 0, s, a);
  if (nfin > 0) hipLaunchKernelGGL(k_ea_nn_fin, dim3((unsigned)nfin), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ea_erow(hipStream_t s, const EnrAsm &a, int nitems, int nfin) {
  if (nitems > 0) hipLaunchKernelGGL(k_ea_erow, dim3((unsigned)nitems), dim3(256), 0, s, a);
  if (nfin > 0) hipLaunchKernelGGL(k_ea_erow_fin, dim3((unsigned)nfin), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ea_ee_reduce(hipStream_t s, const EnrAsm &a, int n_e, int npairs,
                               const int32_t *pair_ij, const int64_t *pair_ptr, const int32_t *pc,
                               double *Hee) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ea_ee_reduce, dim3((unsigned)npairs), dim3(256), 0, s, a, n_e, pair_ij,
                     pair_ptr, pc, Hee);
  return hipGetLastError();
}

hipError_t launch_unit_cols(hipStream_t s, int64_t rows, int N, int64_t ldx, int64_t j0,
                            double *X) {
  if (rows <= 0 || N <= 0) return hipSuccess;
  const int64_t total = rows * N;
  const unsigned nb = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_unit_cols, dim3(nb), dim3(256), 0, s, rows, N, ldx, j0, X);
  return hipGetLastError();
}

}  // namespace cf
