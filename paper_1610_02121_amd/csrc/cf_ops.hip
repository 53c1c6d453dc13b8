// Elemental operator kernels (Sec. IV.D, Sec. V): classical cell products on
// FP64 MFMA, the enriched-cell coupling products (both directions), the
// enrichment-row reductions and the Chebyshev recurrence epilogue.
//
// MFMA fragment layout of v_mfma_f64_16x16x4f64 (wave of 64 lanes):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element r holds D[4 * r + l / 16][l % 16]
#include <algorithm>

#include "cf_kernels.h"

namespace cf {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 d4zero() { d4 z = {0.0, 0.0, 0.0, 0.0}; return z; }

// ---------------------------------------------------------------------------
// Classical cell products of one colour for a single column (the Lanczos
// vectors), Y[dof(e,a)] (=|+=) sum_b H_e[a][b] X[dof(e,b)]: the cell matrix
// streams through once, so the launch is bound by reading it, and the MFMA
// kernel below (one workgroup per CU) would leave that stream latency-bound.
// One 128-thread workgroup per cell (many per CU); thread i forms row i as an
// FMA chain over k = 0..127, reading column i of the symmetric matrix (row k,
// contiguous across the threads) and X[dof(e,k)] from LDS.  Flags and the
// finishing step are those of k_cell_gemm.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NPAD) void k_cell_gemv(
    const double *__restrict__ Hp, const int32_t *__restrict__ dofp,
    const uint8_t *__restrict__ flagp, const int32_t *__restrict__ cells,
    const double *__restrict__ X, int64_t ldx, double *__restrict__ Y, int64_t ldy,
    const CellFinish f) {
  __shared__ double xs[NPAD];
  const int i = threadIdx.x;
  const int cell = cells[blockIdx.x];
  const int d = dofp[(int64_t)cell * NPAD + i];
  const uint8_t fl = flagp[(int64_t)cell * NPAD + i];
  xs[i] = d >= 0 ? X[(int64_t)d * ldx] : 0.0;
  __syncthreads();
  const double *Hc = Hp + (int64_t)cell * NPAD * NPAD + i;
  constexpr int U = 16;
  double acc = 0.0;
#pragma unroll 1
  for (int k0 = 0; k0 < NPAD; k0 += U) {
    double h[U];
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = Hc[(int64_t)(k0 + u) * NPAD];
#pragma unroll
    for (int u = 0; u < U; ++u) acc = fma(h[u], xs[k0 + u], acc);
  }
  if (d < 0) return;
  const double v = acc + ((fl & CELL_FIRST) ? 0.0 : Y[(int64_t)d * ldy]);
  if (f.Out != nullptr && (fl & CELL_FINISH)) {
    const double yp = f.Yp ? f.Yp[(int64_t)d * f.ldyp] : 0.0;
    f.Out[(int64_t)d * f.ldo] = f.c1 * f.dinv[d] * v + f.c2 * xs[i] + f.c3 * yp;
  } else {
    Y[(int64_t)d * ldy] = v;
  }
}

// ---------------------------------------------------------------------------
// Classical cell products for the cells of one colour:
//   Y[dof(e,a)] (=|+=) sum_b H_e[a][b] X[dof(e,b)]
// Two workgroups of 4 waves per cell, each owning 64 output rows; wave w (of
// the cell's 8) owns the 16 output rows [16w, 16w+16) and keeps that slice of
// the (padded, symmetric) cell matrix in registers as MFMA A fragments for the
// whole call.  Columns are walked in tiles of CELL_NT: the next tile's
// gathered X rows and old Y values are loaded into registers (two alternating
// sets for Y) during this tile's MFMA loop, so their latency overlaps the
// matrix work; the current tile sits in LDS, and a tile's results are stored
// during the next tile (see the note at the stores).  Dirichlet and
// padding rows are zero.  Cells of one colour share no DOF, so the
// read-modify-write of Y is race free; the first cell (in launch order) to
// touch a DOF writes instead of adding.
//
// With a finishing step f (f.Out != null), a row whose flag marks the last
// touch of a DOF outside the enriched region is complete here and takes the
// Chebyshev recurrence at once instead of being stored in Y:
//   Out[d] = c1 dinv[d] (H X)[d] + c2 X[d] + c3 Yp[d]
// (X[d] is read from the tile in LDS).  Those rows of Y are left untouched.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void k_cell_gemm(
    const double *__restrict__ Hp, const int32_t *__restrict__ dofp,
    const uint8_t *__restrict__ flagp, const int32_t *__restrict__ cells, int ncells,
    const double *__restrict__ X, int64_t ldx, double *__restrict__ Y, int64_t ldy, int N,
    const CellFinish f) {
  constexpr int NT = CELL_NT;
  constexpr int LDX = NT + 16;
  constexpr int PF = NPAD * NT / 256;        // gathered doubles per thread per tile
  constexpr int RPP = 256 / NT;              // gathered rows per pass
  __shared__ double xs[NPAD * LDX];
  __shared__ int32_t sdof[NPAD];
  __shared__ uint8_t sflag[NPAD];

  // workgroup id -> (cell, half): the two halves of a cell are 8 ids apart,
  // so they run on the same XCD and share its L2 for the gathered rows
  const int id = blockIdx.x;
  const int ci = (id >> 4) * 8 + (id & 7), half = (id >> 3) & 1;
  if (ci >= ncells) return;               // uniform for the workgroup
  const int tid = threadIdx.x, lane = tid & 63, w = (tid >> 6) + 4 * half;
  const int li = lane & 15, kq = lane >> 4;
  const int cell = cells[ci];
  if (tid < NPAD) {
    sdof[tid] = dofp[(int64_t)cell * NPAD + tid];
    sflag[tid] = flagp[(int64_t)cell * NPAD + tid];
  }
  // A[i][k] = H[i][k] = H[k][i]: lane reads H[4ks + kq][16w + li] (contiguous)
  const double *Hc = Hp + (int64_t)cell * NPAD * NPAD;
  double a[32];
#pragma unroll
  for (int ks = 0; ks < 32; ++ks) a[ks] = Hc[(4 * ks + kq) * NPAD + 16 * w + li];
  __syncthreads();

  // gathered X rows: the loads are unconditional (Dirichlet rows and columns
  // past N clamped into the block) and their values untouched until the LDS
  // store, where they are masked
  const int gj = tid % NT, gr = tid / NT;
  int64_t gd[PF];
  bool gok[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    const int d = sdof[gr + p * RPP];
    gok[p] = d >= 0;
    gd[p] = d >= 0 ? d : 0;
  }
  double pf[PF];
  auto gather = [&](int c) {
    const int col = min(c + gj, N - 1);
#pragma unroll
    for (int p = 0; p < PF; ++p) pf[p] = X[gd[p] * ldx + col];
  };
  gather(0);
  const bool finish = f.Out != nullptr;
  int od[4];
  bool ofirst[4], ofin[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * w + kq + 4 * r;
    od[r] = sdof[row];
    ofirst[r] = (sflag[row] & CELL_FIRST) != 0;
    ofin[r] = finish && od[r] >= 0 && (sflag[row] & CELL_FINISH) != 0;
  }

  // the scaled inverse mass of the finishing rows, read once
  double dv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) dv[r] = ofin[r] ? f.c1 * f.dinv[od[r]] : 0.0;

  // old Y (and Yp of finishing rows) of a tile, loaded one tile ahead into
  // one of two register sets
  auto load_y = [&](double (&yo)[4], double (&yp)[4], int c) {
    const bool cv = c + li < N;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      yo[r] = (od[r] >= 0 && !ofirst[r] && cv) ? Y[(int64_t)od[r] * ldy + c + li] : 0.0;
      yp[r] = (ofin[r] && f.Yp && cv) ? f.Yp[(int64_t)od[r] * f.ldyp + c + li] : 0.0;
    }
  };
  // A tile's results are stored during the next tile, after that tile's
  // gathered rows have gone to LDS: global stores and loads pending together
  // make the wave wait for all of its memory operations, so a store issued
  // at the end of a tile would hold up the next tile's LDS fill by its own
  // latency.  Issued one tile later they have a whole MFMA loop to complete.
  double out[4];
  auto store_out = [&](int c0) {
    if (c0 + li >= N) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (od[r] < 0) continue;
      if (ofin[r])
        f.Out[(int64_t)od[r] * f.ldo + c0 + li] = out[r];
      else
        Y[(int64_t)od[r] * ldy + c0 + li] = out[r];
    }
  };
  auto tile = [&](double (&yo)[4], double (&yp)[4], double (&yo2)[4], double (&yp2)[4],
                  int c0) {
#pragma unroll
    for (int p = 0; p < PF; ++p) xs[(gr + p * RPP) * LDX + gj] = (gok[p] && c0 + gj < N) ? pf[p] : 0.0;
    if (c0 > 0) store_out(c0 - NT);
    __syncthreads();
    const int c1 = c0 + NT;
    if (c1 < N) {
      gather(c1);
      load_y(yo2, yp2, c1);
    }
    d4 acc = d4zero();
#pragma unroll
    for (int ks = 0; ks < 32; ++ks) acc = mfma_f64(a[ks], xs[(4 * ks + kq) * LDX + li], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double v = acc[r] + yo[r];
      const double xk = xs[(16 * w + kq + 4 * r) * LDX + li];
      out[r] = ofin[r] ? dv[r] * v + f.c2 * xk + f.c3 * yp[r] : v;
    }
    __syncthreads();
  };
  double ya[4], pa[4], yb[4], pb[4];
  load_y(ya, pa, 0);
  int clast = 0;
  for (int c0 = 0; c0 < N; c0 += 2 * NT) {
    tile(ya, pa, yb, pb, c0);
    clast = c0;
    if (c0 + NT < N) {
      tile(yb, pb, ya, pa, c0 + NT);
      clast = c0 + NT;
    }
  }
  store_out(clast);
}

hipError_t launch_cell_gemm(hipStream_t s, const double *Hp, const int32_t *dofp,
                            const uint8_t *flagp, const int32_t *cells, int ncells,
                            const double *X, int64_t ldx, double *Y, int64_t ldy, int N,
                            const CellFinish &f) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  if (N == 1) {
    hipLaunchKernelGGL(k_cell_gemv, dim3(ncells), dim3(NPAD), 0, s, Hp, dofp, flagp, cells, X,
                       ldx, Y, ldy, f);
    return hipGetLastError();
  }
  // two workgroups (each 64 output rows) per cell, ids laid out by k_cell_gemm
  const int nblk = 16 * ((ncells + 7) / 8);
  hipLaunchKernelGGL(k_cell_gemm, dim3(nblk), dim3(256), 0, s, Hp, dofp, flagp, cells, ncells, X,
                     ldx, Y, ldy, N, f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Enriched-cell coupling partials (one workgroup per group of at most 4
// output row blocks of an enriched cell, walking column tiles of 16):
//   P[k0+k] = cH * sum_a H^ec_e[k][a] X[dof(e,a)]
//           + cM * sum_a M^ec_e[k][a] s(dof) R[dof(e,a)]
// The cell blocks are stored transposed, [NPAD][nap] with nap = the cell's
// enrichment count padded to 16, so A-fragment loads are contiguous.  The
// blocks are read from memory once per call: every wave keeps its A fragments
// in registers while the column tiles stream by (cells with more than 64
// enrichment functions take one workgroup per 64 output rows, placed on one
// XCD so that they gather the cell's rows through one L2).  The next tile's
// gathered rows are loaded into registers during the current tile's MFMAs.
// Either term is skipped when its input block is null.
// ---------------------------------------------------------------------------
// 8 waves split between the cell's 16-row output blocks and the 128 k (local
// nodes): with B = 4 blocks per group (cells with 3 or more blocks) wave w
// takes block 4g + (w & 3) of group g and k half w >> 2; cells with 2 blocks
// take B = 2 blocks and k quarters, cells with one block B = 1 and k eighths,
// so every wave (and every SIMD) carries products whatever the block count.
// A wave keeps the A fragments of both terms for its k part in registers
// while the column tiles stream by; the KP = 8 / B partial sums are added
// through LDS in k-part order.  The gathered rows of a tile are loaded one
// tile ahead into registers.
template <int B>
__device__ __forceinline__ void enr_part_body(
    const double *__restrict__ ht, const double *__restrict__ mt, int nap, int nmb, int na,
    int64_t k0, const int (&gd)[4], const double (&gsc)[4], const double *__restrict__ X,
    int64_t ldx, double cH, const double *__restrict__ R, int64_t ldr, double cM,
    double *__restrict__ P, int64_t ldp, int cbeg, int cend, int g, double *xs, double *rsm,
    double *xch) {
  constexpr int PT = 16, LDX = PT + 1, PF = 4, RPP = 32;
  constexpr int KP = 8 / B, KS = NPAD / KP, NKS = KS / 4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int wb = w % B, h = w / B;
  const int gj = tid % PT, gr = tid / PT;
  {
    const int mb = B * g + wb;
    const bool act = mb < nmb;
    double aH[NKS], aM[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int64_t off = (int64_t)(KS * h + 4 * ks + kq) * nap + 16 * mb + li;
      aH[ks] = (act && ht) ? ht[off] : 0.0;
      aM[ks] = (act && mt) ? mt[off] : 0.0;
    }
    // the gathered rows of the next tile, loaded during this tile's MFMAs.
    // The loads are unconditional (row and column clamped into the block) and
    // nothing touches their values before the LDS store, where the masking and
    // the R scaling are applied.  A tile's partial sums are stored during the
    // next tile, after its LDS fill: pending global stores make the wave wait
    // for all of its memory operations, so stores issued at the end of a tile
    // would hold up the next fill by their own latency.
    double qx[PF], qr[PF], out[4];
    auto gather = [&](int c) {
      const int col = min(c + gj, cend - 1);
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int64_t row = gd[p] >= 0 ? gd[p] : 0;
        if (X) qx[p] = X[row * ldx + col];
        if (R) qr[p] = R[row * ldr + col];
      }
    };
    auto store_out = [&](int c0) {
      if (act && h == 0 && c0 + li < cend) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int orow = 16 * mb + kq + 4 * r;
          if (orow < na) P[(k0 + orow) * ldp + c0 + li] = out[r];
        }
      }
    };
    gather(cbeg);
    for (int c0 = cbeg; c0 < cend; c0 += PT) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const bool v = gd[p] >= 0 && c0 + gj < cend;
        xs[(gr + p * RPP) * LDX + gj] = (X && v) ? qx[p] : 0.0;
        rsm[(gr + p * RPP) * LDX + gj] = (R && v) ? qr[p] * gsc[p] : 0.0;
      }
      if (c0 > cbeg) store_out(c0 - PT);
      __syncthreads();
      if (c0 + PT < cend) gather(c0 + PT);
      d4 acc = d4zero();
      if (act) {
        d4 accH = d4zero(), accM = d4zero();
        if (ht) {
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks)
            accH = mfma_f64(aH[ks], xs[(KS * h + 4 * ks + kq) * LDX + li], accH);
        }
        if (mt) {
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks)
            accM = mfma_f64(aM[ks], rsm[(KS * h + 4 * ks + kq) * LDX + li], accM);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = cH * accH[r] + cM * accM[r];
        if (h > 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) xch[(((h - 1) * B + wb) * 4 + r) * 64 + lane] = acc[r];
        }
      }
      __syncthreads();
      if (act && h == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double v = acc[r];
#pragma unroll
          for (int q = 1; q < KP; ++q) v += xch[(((q - 1) * B + wb) * 4 + r) * 64 + lane];
          out[r] = v;
        }
      }
    }
    store_out(cbeg + PT * ((cend - cbeg - 1) / PT));
    __syncthreads();
  }
}

// A workgroup takes one item: a group of (at most) 4 output row blocks of one
// enriched cell, item = (position in `cells`) * 32 + group; -1 items are
// padding.  blockIdx.y picks one of gridDim.y contiguous ranges of column
// tiles.
__global__ __launch_bounds__(512, 2) void k_enr_part(
    const double *__restrict__ HT, const double *__restrict__ MT,
    const int64_t *__restrict__ toff, const int32_t *__restrict__ tld,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ dofp,
    const int32_t *__restrict__ cells, const int32_t *__restrict__ items,
    const double *__restrict__ X, int64_t ldx, double cH,
    const double *__restrict__ R, int64_t ldr, const double *__restrict__ rs, double cM,
    double *__restrict__ P, int64_t ldp, int N) {
  constexpr int PT = 16, LDX = PT + 1, PF = 4, RPP = 32;
  __shared__ double xs[NPAD * LDX];
  __shared__ double rsm[NPAD * LDX];
  __shared__ double xch[7 * 4 * 64];      // partial sums of k parts 1..KP-1
  const int tid = threadIdx.x;
  const int item = items[blockIdx.x];
  if (item < 0) return;                  // uniform for the workgroup
  const int cell = cells[item >> 5], grp = item & 31;
  const int ntile = (N + PT - 1) / PT;
  const int cbeg = PT * ((ntile * (int)blockIdx.y) / (int)gridDim.y);
  const int cend = min(N, PT * ((ntile * ((int)blockIdx.y + 1)) / (int)gridDim.y));
  const int gr = tid / PT;
  int gd[PF];
  double gsc[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    gd[p] = dofp[(int64_t)cell * NPAD + gr + p * RPP];
    gsc[p] = (rs && gd[p] >= 0) ? rs[gd[p]] : 1.0;
  }
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  const int nap = tld[cell];
  const int nmb = nap >> 4;
  const double *ht = X ? HT + toff[cell] : nullptr;
  const double *mt = R ? MT + toff[cell] : nullptr;
  if (cbeg >= cend) return;              // uniform for the workgroup
  if (nmb >= 3)
    enr_part_body<4>(ht, mt, nap, nmb, na, k0, gd, gsc, X, ldx, cH, R, ldr, cM, P, ldp, cbeg, cend,
                     grp, xs, rsm, xch);
  else if (nmb == 2)
    enr_part_body<2>(ht, mt, nap, nmb, na, k0, gd, gsc, X, ldx, cH, R, ldr, cM, P, ldp, cbeg, cend,
                     0, xs, rsm, xch);
  else
    enr_part_body<1>(ht, mt, nap, nmb, na, k0, gd, gsc, X, ldx, cH, R, ldr, cM, P, ldp, cbeg, cend,
                     0, xs, rsm, xch);
}

// Single-column form (the Lanczos vectors): the coupling blocks stream
// through once, so one 256-thread workgroup per enriched cell (many per CU)
// with thread k forming output row k from row a of the transposed blocks
// (contiguous across the threads) and the gathered X, s R values in LDS; the
// two 64-node halves are summed separately and added as in k_enr_part.
__global__ __launch_bounds__(256) void k_enr_part_vec(
    const double *__restrict__ HT, const double *__restrict__ MT,
    const int64_t *__restrict__ toff, const int32_t *__restrict__ tld,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ dofp,
    const int32_t *__restrict__ cells, const double *__restrict__ X, int64_t ldx, double cH,
    const double *__restrict__ R, int64_t ldr, const double *__restrict__ rs, double cM,
    double *__restrict__ P, int64_t ldp) {
  __shared__ double xg[NPAD], rg[NPAD];
  const int tid = threadIdx.x;
  const int cell = cells[blockIdx.x];
  if (tid < NPAD) {
    const int d = dofp[(int64_t)cell * NPAD + tid];
    xg[tid] = (X && d >= 0) ? X[(int64_t)d * ldx] : 0.0;
    rg[tid] = (R && d >= 0) ? R[(int64_t)d * ldr] * (rs ? rs[d] : 1.0) : 0.0;
  }
  __syncthreads();
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  const int nap = tld[cell];
  const double *ht = X ? HT + toff[cell] : nullptr;
  const double *mt = R ? MT + toff[cell] : nullptr;
  for (int k = tid; k < na; k += 256) {
    double acc = 0.0;
    for (int h = 0; h < 2; ++h) {
      double sh = 0.0, sm = 0.0;
      if (ht) {
#pragma unroll 16
        for (int a = 64 * h; a < 64 * h + 64; ++a) sh = fma(ht[(int64_t)a * nap + k], xg[a], sh);
      }
      if (mt) {
#pragma unroll 16
        for (int a = 64 * h; a < 64 * h + 64; ++a) sm = fma(mt[(int64_t)a * nap + k], rg[a], sm);
      }
      const double part = cH * sh + cM * sm;
      acc = h == 0 ? part : acc + part;
    }
    P[(k0 + k) * ldp] = acc;
  }
}

hipError_t launch_enr_part(hipStream_t s, const double *HT, const double *MT, const int64_t *toff,
                           const int32_t *tld, const int64_t *eptr, const int32_t *dofp,
                           const int32_t *cells, int ncells, const int32_t *items, int nitems,
                           const double *X, int64_t ldx, double cH, const double *R, int64_t ldr,
                           const double *rs, double cM, double *P, int64_t ldp, int N) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  if (N == 1) {
    hipLaunchKernelGGL(k_enr_part_vec, dim3(ncells), dim3(256), 0, s, HT, MT, toff, tld, eptr,
                       dofp, cells, X, ldx, cH, R, ldr, rs, cM, P, ldp);
    return hipGetLastError();
  }
  // one column range per item (splitting the columns over 2-4 workgroups per
  // cell measured slower on the 30-atom workload: the blocks are re-read)
  hipLaunchKernelGGL(k_enr_part, dim3(nitems, 1), dim3(512), 0, s, HT, MT, toff, tld, eptr, dofp,
                     cells, items, X, ldx, cH, R, ldr, rs, cM, P, ldp, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transposed coupling products of the enriched cells, into a cell-local buffer
// (one workgroup per enriched cell, walking column tiles of 16; no
// read-modify-write):
//   Q[128 e' + a] = sum_k (cU H^ec_e[k][a] U[idx_k] + cV M^ec_e[k][a] V[idx_k])
// e' is the position of the cell in the enriched-cell list, a its local node.
// The enrichment functions of the cell are taken in chunks of 64 (16 or 32
// for cells with at most that many).  Two workgroups of 4 waves share a cell
// (blockIdx.y picks 64 of its 128 local nodes): wave w keeps the A fragments of
// rows 16w .. 16w+16 of both transposed blocks for the chunk in registers
// while the column tiles stream by (the blocks are read from memory once per
// call); the gathered rows cU U[idx_k], cV V[idx_k] of the chunk pass through
// LDS, loaded one tile ahead into registers; chunks after the first add into
// Q.  Either term is skipped when its input is null.  The epilogue sums, for
// each classical DOF, the (at most 8) Q rows of the enriched cells that
// contain it.
// ---------------------------------------------------------------------------
// Cells with at most 16 or 32 enrichment functions take chunks of that size
// (KC = 16 or 32), so their waves run only the k steps that carry products.
template <int KC>
__device__ __forceinline__ void enr_q_body(
    const double *__restrict__ Hec, const double *__restrict__ Mec, int64_t k0, int na,
    const int32_t *__restrict__ eidx, const double *__restrict__ U, int64_t ldu, double cU,
    const double *__restrict__ V, int64_t ldv, double cV, double *__restrict__ qb, int64_t ldq,
    int N, double *zu, double *zv, double *qs) {
  constexpr int PT = 16, LDZ = 16, KS = KC / 4;
  constexpr int GR = 256 / PT;             // gathered rows per pass
  constexpr int GV = (KC + GR - 1) / GR;   // passes per term and tile
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = (tid >> 6) + 4 * (int)blockIdx.y;   // 16-row block of the 128 local nodes
  const int li = lane & 15, kq = lane >> 4;
  const int gj = tid % PT, gk = tid / PT;   // gather: column gj, rows gk + GR p
  for (int kc = 0; kc < na; kc += KC) {
    double aH[KS], aM[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = kc + 4 * ks + kq;
      const bool v = k < na;
      const int64_t off = (k0 + (v ? k : 0)) * NPAD + 16 * w + li;
      aH[ks] = (U && v) ? Hec[off] : 0.0;
      aM[ks] = (V && v) ? Mec[off] : 0.0;
    }
    int64_t gal[GV];
    bool gv[GV];
#pragma unroll
    for (int p = 0; p < GV; ++p) {
      const int k = kc + gk + GR * p;
      gv[p] = gk + GR * p < KC && k < na;
      gal[p] = gv[p] ? eidx[k0 + k] : 0;
    }
    // the next tile's gathered rows, loaded during this tile's MFMAs; the
    // loads are unconditional (column clamped) and their values untouched
    // until the LDS store.  A tile's Q values are parked in LDS (each lane
    // reads back only what it wrote) and stored to memory during the next
    // tile, after its LDS fill: pending global stores make the wave wait for
    // all of its memory operations, so stores issued at the end of a tile
    // would hold up the next fill by their own latency.
    double pu[GV], pv[GV];
    auto gather = [&](int c) {
      const int col = min(c + gj, N - 1);
#pragma unroll
      for (int p = 0; p < GV; ++p) {
        if (U) pu[p] = U[gal[p] * ldu + col];
        if (V) pv[p] = V[gal[p] * ldv + col];
      }
    };
    auto store_q = [&](int c0) {
      if (c0 + li < N) {
        double *q = qb + c0 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * w + kq + 4 * r;
          q[(int64_t)row * ldq] = qs[row * PT + li];
        }
      }
    };
    gather(0);
    for (int c0 = 0; c0 < N; c0 += PT) {
#pragma unroll
      for (int p = 0; p < GV; ++p) {
        if (gk + GR * p < KC) {
          const bool v = gv[p] && c0 + gj < N;
          zu[(gk + GR * p) * LDZ + gj] = (U && v) ? cU * pu[p] : 0.0;
          zv[(gk + GR * p) * LDZ + gj] = (V && v) ? cV * pv[p] : 0.0;
        }
      }
      if (c0 > 0) store_q(c0 - PT);
      __syncthreads();
      if (c0 + PT < N) gather(c0 + PT);
      // chunks after the first add into Q: its old values, loaded before the
      // products so that their latency overlaps them
      double qo[4];
      if (kc > 0) {
        const double *q = qb + min(c0 + li, N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) qo[r] = q[(int64_t)(16 * w + kq + 4 * r) * ldq];
      }
      d4 acc = d4zero();
      if (U) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc = mfma_f64(aH[ks], zu[(4 * ks + kq) * LDZ + li], acc);
      }
      if (V) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc = mfma_f64(aM[ks], zv[(4 * ks + kq) * LDZ + li], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        qs[(16 * w + kq + 4 * r) * PT + li] = acc[r] + (kc > 0 ? qo[r] : 0.0);
      __syncthreads();
    }
    store_q(PT * ((N - 1) / PT));
  }
}

__global__ __launch_bounds__(256, 2) void k_enr_q(
    const double *__restrict__ Hec, const double *__restrict__ Mec,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ eidx,
    const int32_t *__restrict__ cells, const int32_t *__restrict__ order,
    const double *__restrict__ U, int64_t ldu, double cU,
    const double *__restrict__ V, int64_t ldv, double cV, double *__restrict__ Q, int64_t ldq,
    int N) {
  constexpr int PT = 16, LDZ = 16, KC = 64;
  __shared__ double zu[KC * LDZ];
  __shared__ double zv[KC * LDZ];
  __shared__ double qs[NPAD * PT];         // a tile's Q values until their store
  const int tid = threadIdx.x;
  const int pos = order ? order[blockIdx.x] : (int)blockIdx.x;   // position in the cell list
  const int cell = cells[pos];
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  double *qb = Q + ((int64_t)pos * NPAD) * ldq;
  if (na > 32)
    enr_q_body<64>(Hec, Mec, k0, na, eidx, U, ldu, cU, V, ldv, cV, qb, ldq, N, zu, zv, qs);
  else if (na > 16)
    enr_q_body<32>(Hec, Mec, k0, na, eidx, U, ldu, cU, V, ldv, cV, qb, ldq, N, zu, zv, qs);
  else if (na > 0)
    enr_q_body<16>(Hec, Mec, k0, na, eidx, U, ldu, cU, V, ldv, cV, qb, ldq, N, zu, zv, qs);
  if (na == 0) {
    // no enrichment functions: the workgroup's 64 buffer rows are zero
    for (int c0 = 0; c0 < N; c0 += PT)
      for (int idx = tid; idx < 64 * PT; idx += 256) {
        const int a = 64 * (int)blockIdx.y + idx / PT, j = idx % PT;
        if (c0 + j < N) qb[(int64_t)a * ldq + c0 + j] = 0.0;
      }
  }
}

// Single-column form of k_enr_q: one 128-thread workgroup per enriched cell,
// thread a forming Q row a from row k of the blocks (contiguous across the
// threads) and the gathered cU U[idx_k], cV V[idx_k] in LDS, in chunks of 64
// enrichment functions (each chunk's sum added to the previous ones, as the
// MFMA kernel adds into Q); Q is written once.
__global__ __launch_bounds__(NPAD) void k_enr_q_vec(
    const double *__restrict__ Hec, const double *__restrict__ Mec,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ eidx,
    const int32_t *__restrict__ cells, const int32_t *__restrict__ order,
    const double *__restrict__ U, int64_t ldu, double cU,
    const double *__restrict__ V, int64_t ldv, double cV, double *__restrict__ Q, int64_t ldq) {
  constexpr int KC = 64;
  __shared__ double zu[KC], zv[KC];
  const int a = threadIdx.x;
  const int pos = order ? order[blockIdx.x] : (int)blockIdx.x;
  const int cell = cells[pos];
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  double acc = 0.0;
  for (int kc = 0; kc < na; kc += KC) {
    const int kn = min(KC, na - kc);
    if (a < KC) {
      const bool v = a < kn;
      const int64_t al = v ? eidx[k0 + kc + a] : 0;
      zu[a] = (U && v) ? cU * U[al * ldu] : 0.0;
      zv[a] = (V && v) ? cV * V[al * ldv] : 0.0;
    }
    __syncthreads();
    double sc = 0.0;
    if (U) {
      for (int k = 0; k < kn; ++k) sc = fma(Hec[(k0 + kc + k) * NPAD + a], zu[k], sc);
    }
    if (V) {
      for (int k = 0; k < kn; ++k) sc = fma(Mec[(k0 + kc + k) * NPAD + a], zv[k], sc);
    }
    acc = kc == 0 ? sc : sc + acc;
    __syncthreads();
  }
  Q[((int64_t)pos * NPAD + a) * ldq] = acc;
}

hipError_t launch_enr_q(hipStream_t s, const double *Hec, const double *Mec, const int64_t *eptr,
                        const int32_t *eidx, const int32_t *cells, const int32_t *order,
                        int ncells, int kmax, const double *U, int64_t ldu, double cU,
                        const double *V, int64_t ldv, double cV, double *Q, int64_t ldq, int N) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  (void)kmax;
  if (N == 1) {
    hipLaunchKernelGGL(k_enr_q_vec, dim3(ncells), dim3(NPAD), 0, s, Hec, Mec, eptr, eidx, cells,
                       order, U, ldu, cU, V, ldv, cV, Q, ldq);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_enr_q, dim3(ncells, 2), dim3(256), 0, s, Hec, Mec, eptr, eidx, cells, order, U,
                     ldu, cU, V, ldv, cV, Q, ldq, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Enrichment rows (grid: column tiles of 64 x n_e): fixed-order segmented sum
// of the per-cell partials, plus an optional dense n_e x n_e product and an
// optional scaled extra term.  Deterministic: no atomics.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_enr_reduce(
    int n_e, const int64_t *__restrict__ aptr, const int32_t *__restrict__ alist,
    const double *__restrict__ P, int64_t ldp, double s_p, const double *__restrict__ R0,
    int64_t ldr0, double s_r, const double *__restrict__ Dn, const double *__restrict__ Zd,
    int64_t ldzd, double *__restrict__ out, int64_t ldo, int N) {
  // 4 waves split the partial rows and the dense product into 4 contiguous
  // ranges each (a partition fixed by the sizes), combined in wave order
  __shared__ double part[2][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  const int al = blockIdx.y;
  const bool cv = col < N;
  double sp = 0.0, sd = 0.0;
  // the sums run in index order; the loads of 8 terms are issued before
  // their adds (memory-level parallelism without changing the rounding)
  constexpr int U = 8;
  if (P && cv) {
    const int64_t a0 = aptr[al], a1 = aptr[al + 1], len = a1 - a0;
    const int64_t q0 = a0 + (len * w) / 4, q1 = a0 + (len * (w + 1)) / 4;
    int64_t k = q0;
    for (; k + U <= q1; k += U) {
      double t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) t[u] = P[(int64_t)alist[k + u] * ldp + col];
#pragma unroll
      for (int u = 0; u < U; ++u) sp += t[u];
    }
    for (; k < q1; ++k) sp += P[(int64_t)alist[k] * ldp + col];
  }
  if (Dn && cv) {
    const double *drow = Dn + (int64_t)al * n_e;
    const int b0 = (n_e * w) / 4, b1 = (n_e * (w + 1)) / 4;
    int be = b0;
    for (; be + U <= b1; be += U) {
      double t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) t[u] = Zd[(int64_t)(be + u) * ldzd + col];
#pragma unroll
      for (int u = 0; u < U; ++u) sd += drow[be + u] * t[u];
    }
    for (; be < b1; ++be) sd += drow[be] * Zd[(int64_t)be * ldzd + col];
  }
  part[0][w][lane] = sp;
  part[1][w][lane] = sd;
  __syncthreads();
  if (w == 0 && cv) {
    double acc = 0.0;
    if (P) acc = s_p * (((part[0][0][lane] + part[0][1][lane]) + part[0][2][lane]) + part[0][3][lane]);
    if (R0) acc += s_r * R0[(int64_t)al * ldr0 + col];
    if (Dn) acc += ((part[1][0][lane] + part[1][1][lane]) + part[1][2][lane]) + part[1][3][lane];
    out[(int64_t)al * ldo + col] = acc;
  }
}

hipError_t launch_enr_reduce(hipStream_t s, int n_e, const int64_t *aptr, const int32_t *alist,
                             const double *P, int64_t ldp, double s_p, const double *R0,
                             int64_t ldr0, double s_r, const double *Dn, const double *Zd,
                             int64_t ldzd, double *out, int64_t ldo, int N) {
  if (n_e <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + 63) / 64, n_e);
  hipLaunchKernelGGL(k_enr_reduce, grid, dim3(256), 0, s, n_e, aptr, alist, P, ldp, s_p, R0, ldr0,
                     s_r, Dn, Zd, ldzd, out, ldo, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Epilogue over all n = n_h + n_e rows, or over a list of classical rows and
// the enrichment rows (block: 64 columns x 4 rows):
//   classical row i:  v = dR_i R[i] + dC_i sum_p Q[qidx[p]]   (p over qptr[i]..qptr[i+1];
//                     the rows of the enriched-cell buffer holding DOF i; null
//                     scales mean 1)
//   enrichment row:   v = Ee[i - n_h]
//   Out[i] = c1 v + c2 Yk[i] + c3 Yp[i]       (null Yk / Yp skipped)
// Out may alias R or Yp: each element is read before the same thread writes it.
// ---------------------------------------------------------------------------
// Below EPI_FEW_COLS columns one thread takes one element (rows across the
// lanes) instead of 64 lanes sharing a row; the arithmetic of an element is
// the same in both mappings.
constexpr int EPI_FEW_COLS = 16;

__global__ __launch_bounds__(256) void k_epilogue(const EpiArgs g) {
  // rows: all n_h + n_e rows, or the listed classical rows followed by the n_e
  // enrichment rows
  const int64_t ncls = g.rows ? g.nrows : g.n_h;
  const int64_t nt = ncls + g.n_e;
  if (g.N < EPI_FEW_COLS) {
    const int64_t total = nt * g.N;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.y * 64 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
      const int64_t t = e / g.N;
      const int j = (int)(e - t * g.N);
      const bool cls = t < ncls;
      const int64_t i = cls ? (g.rows ? (int64_t)g.rows[t] : t) : g.n_h + (t - ncls);
      double v;
      if (cls) {
        const double dr = g.dR ? g.dR[i] : 1.0;
        v = dr * g.R[i * g.ldr + j];
        if (g.qptr) {
          const int p0 = g.qptr[i], p1 = g.qptr[i + 1];
          if (p1 > p0) {
            const double dc = g.dC ? g.dC[i] : 1.0;
            double sq = 0.0;
            for (int p = p0; p < p1; ++p) sq += g.Q[(int64_t)g.qidx[p] * g.ldq + j];
            v += dc * sq;
          }
        }
      } else {
        v = g.Ee[(i - g.n_h) * g.lde + j];
      }
      v *= g.c1;
      if (g.Yk) v += g.c2 * g.Yk[i * g.ldyk + j];
      if (g.Yp) v += g.c3 * g.Yp[i * g.ldyp + j];
      g.Out[i * g.ldo + j] = v;
    }
    return;
  }
  for (int64_t t = (int64_t)blockIdx.x * 4 + threadIdx.y; t < nt; t += (int64_t)gridDim.x * 4) {
    const bool cls = t < ncls;
    const int64_t i = cls ? (g.rows ? (int64_t)g.rows[t] : t) : g.n_h + (t - ncls);
    double dr = 1.0, dc = 1.0;
    int p0 = 0, p1 = 0;
    if (cls) {
      if (g.dR) dr = g.dR[i];
      if (g.dC) dc = g.dC[i];
      if (g.qptr) { p0 = g.qptr[i]; p1 = g.qptr[i + 1]; }
    }
    for (int j = threadIdx.x; j < g.N; j += 64) {
      double v;
      if (cls) {
        v = dr * g.R[i * g.ldr + j];
        if (p1 > p0) {
          double sq = 0.0;
          for (int p = p0; p < p1; ++p) sq += g.Q[(int64_t)g.qidx[p] * g.ldq + j];
          v += dc * sq;
        }
      } else {
        v = g.Ee[(i - g.n_h) * g.lde + j];
      }
      v *= g.c1;
      if (g.Yk) v += g.c2 * g.Yk[i * g.ldyk + j];
      if (g.Yp) v += g.c3 * g.Yp[i * g.ldyp + j];
      g.Out[i * g.ldo + j] = v;
    }
  }
}

// The same epilogue with two columns per lane (16-byte loads and stores),
// the buffer-row offsets of a DOF (at most EPI_QMAX) held in registers and
// all loads of an element pair issued before its sums.  Used when every
// block pointer is 16-byte aligned and every leading dimension even; the
// arithmetic of each element is that of k_epilogue (same terms, same order).
constexpr int EPI_QMAX = 8;

__global__ __launch_bounds__(256) void k_epilogue_v2(const EpiArgs g) {
  const int64_t ncls = g.rows ? g.nrows : g.n_h;
  const int64_t nt = ncls + g.n_e;
  for (int64_t t = (int64_t)blockIdx.x * 4 + threadIdx.y; t < nt; t += (int64_t)gridDim.x * 4) {
    const bool cls = t < ncls;
    const int64_t i = cls ? (g.rows ? (int64_t)g.rows[t] : t) : g.n_h + (t - ncls);
    double dr = 1.0, dc = 1.0;
    int nq = 0;
    int64_t qo[EPI_QMAX];
    if (cls) {
      if (g.dR) dr = g.dR[i];
      if (g.dC) dc = g.dC[i];
      if (g.qptr) {
        const int p0 = g.qptr[i];
        nq = g.qptr[i + 1] - p0;
#pragma unroll
        for (int u = 0; u < EPI_QMAX; ++u) qo[u] = u < nq ? (int64_t)g.qidx[p0 + u] * g.ldq : 0;
      }
    }
    const double *src = cls ? g.R + i * g.ldr : g.Ee + (i - g.n_h) * g.lde;
    for (int j = 2 * threadIdx.x; j < g.N; j += 128) {
      if (j + 1 < g.N) {
        const double2 r = *reinterpret_cast<const double2 *>(src + j);
        double2 q[EPI_QMAX];
#pragma unroll
        for (int u = 0; u < EPI_QMAX; ++u)
          q[u] = u < nq ? *reinterpret_cast<const double2 *>(g.Q + qo[u] + j) : double2{0.0, 0.0};
        const double2 yk = g.Yk ? *reinterpret_cast<const double2 *>(g.Yk + i * g.ldyk + j)
                                : double2{0.0, 0.0};
        const double2 yp = g.Yp ? *reinterpret_cast<const double2 *>(g.Yp + i * g.ldyp + j)
                                : double2{0.0, 0.0};
        double v0 = cls ? dr * r.x : r.x, v1 = cls ? dr * r.y : r.y;
        if (nq > 0) {
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int u = 0; u < EPI_QMAX; ++u)
            if (u < nq) { s0 += q[u].x; s1 += q[u].y; }
          v0 += dc * s0;
          v1 += dc * s1;
        }
        v0 *= g.c1;
        v1 *= g.c1;
        if (g.Yk) { v0 += g.c2 * yk.x; v1 += g.c2 * yk.y; }
        if (g.Yp) { v0 += g.c3 * yp.x; v1 += g.c3 * yp.y; }
        *reinterpret_cast<double2 *>(g.Out + i * g.ldo + j) = double2{v0, v1};
      } else {
        double v = cls ? dr * src[j] : src[j];
        if (nq > 0) {
          double sq = 0.0;
#pragma unroll
          for (int u = 0; u < EPI_QMAX; ++u)
            if (u < nq) sq += g.Q[qo[u] + j];
          v += dc * sq;
        }
        v *= g.c1;
        if (g.Yk) v += g.c2 * g.Yk[i * g.ldyk + j];
        if (g.Yp) v += g.c3 * g.Yp[i * g.ldyp + j];
        g.Out[i * g.ldo + j] = v;
      }
    }
  }
}

static bool al16(const void *p, int64_t ld) {
  return p == nullptr || (((uintptr_t)p & 15) == 0 && (ld & 1) == 0);
}

hipError_t launch_epilogue(hipStream_t s, const EpiArgs &g) {
  const int64_t n = (g.rows ? g.nrows : g.n_h) + g.n_e;
  if (n <= 0 || g.N <= 0) return hipSuccess;
  int64_t blocks = g.N < EPI_FEW_COLS ? (n * g.N + 255) / 256 : (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  const bool v2 = g.N >= EPI_FEW_COLS && g.qmax <= EPI_QMAX && al16(g.R, g.ldr) &&
                  al16(g.Q, g.ldq) && al16(g.Ee, g.lde) && al16(g.Yk, g.ldyk) &&
                  al16(g.Yp, g.ldyp) && al16(g.Out, g.ldo);
  if (v2)
    hipLaunchKernelGGL(k_epilogue_v2, dim3((unsigned)blocks), dim3(64, 4), 0, s, g);
  else
    hipLaunchKernelGGL(k_epilogue, dim3((unsigned)blocks), dim3(64, 4), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Setup: node-major coupling values.  For the enriched cells of one colour,
// thread a of cell e adds every H^ec_e[k][a], M^ec_e[k][a] into the CSR slot
// of (dof(e,a), alpha_k).  Cells of one colour share no DOF and one cell's
// alphas are distinct, so no two threads of a launch hit the same slot.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_csr_fill(const double *__restrict__ Hec,
                                                  const double *__restrict__ Mec,
                                                  const int64_t *__restrict__ eptr,
                                                  const int32_t *__restrict__ smap,
                                                  const int32_t *__restrict__ cells, double *hv,
                                                  double *mv) {
  const int cell = cells[blockIdx.x];
  const int a = threadIdx.x;
  for (int64_t k = eptr[cell]; k < eptr[cell + 1]; ++k) {
    const int32_t slot = smap[k * NPAD + a];
    if (slot < 0) continue;
    hv[slot] += Hec[k * NPAD + a];
    mv[slot] += Mec[k * NPAD + a];
  }
}

hipError_t launch_csr_fill(hipStream_t s, const double *Hec, const double *Mec,
                           const int64_t *eptr, const int32_t *smap, const int32_t *cells,
                           int ncells, double *hv, double *mv) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_csr_fill, dim3(ncells), dim3(NPAD), 0, s, Hec, Mec, eptr, smap, cells, hv,
                     mv);
  return hipGetLastError();
}

// Dense coupling rows of the enriched region, scaled by D^-1/2:
//   BM[r][ci[p]] = mv[p] / sqrt(D_i),  BH[r][ci[p]] = hv[p] / sqrt(D_i),  i = regrow[r]
__global__ __launch_bounds__(256) void k_csr_dense(int64_t nreg, const int32_t *__restrict__ regrow,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ ci,
                                                   const double *__restrict__ hv,
                                                   const double *__restrict__ mv,
                                                   const double *__restrict__ dinv, double *BM,
                                                   double *BH, int64_t ldb) {
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < nreg;
       r += (int64_t)gridDim.x * 256) {
    const int i = regrow[r];
    const double sc = sqrt(dinv[i]);
    for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      BM[r * ldb + ci[p]] = mv[p] * sc;
      BH[r * ldb + ci[p]] = hv[p] * sc;
    }
  }
}

hipError_t launch_csr_dense(hipStream_t s, int64_t nreg, const int32_t *regrow,
                            const int32_t *rowptr, const int32_t *ci, const double *hv,
                            const double *mv, const double *dinv, double *BM, double *BH,
                            int64_t ldb) {
  if (nreg <= 0) return hipSuccess;
  int64_t blocks = (nreg + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_csr_dense, dim3((unsigned)blocks), dim3(256), 0, s, nreg, regrow, rowptr, ci,
                     hv, mv, dinv, BM, BH, ldb);
  return hipGetLastError();
}

}  // namespace cf
