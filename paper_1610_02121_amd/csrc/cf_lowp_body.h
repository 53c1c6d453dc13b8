// Device bodies of the reduced-precision (FP32 / BF16-input) operator
// kernels, shared by the single-problem kernels (cf_lowp.hip) and the batched
// kernels (cf_batch.hip), so that both compute bit-identical results.  Each
// body takes its work item (cell, row block) explicitly instead of reading
// blockIdx.
//
// MFMA fragment layouts (wave of 64 lanes, l = lane):
//   v_mfma_f32_16x16x4f32:   A[l%16][l/16], B[l/16][l%16], D[4(l/16)+r][l%16]
//   v_mfma_f32_16x16x32_bf16: A[l%16][8(l/16)+i], B[8(l/16)+i][l%16] (i < 8),
//                             D[4(l/16)+r][l%16]
#pragma once

#include "cf_kernels.h"

namespace cf {
namespace lowp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 f4zero() { f4 z = {0.f, 0.f, 0.f, 0.f}; return z; }

// max of |v| that keeps NaN (a NaN compares above every finite value and Inf
// as unsigned float bits)
__device__ __forceinline__ float absmax(float m, float v) {
  const float a = fabsf(v);
  return (a > m || a != a) ? a : m;
}
// Block-wide absmax of m, then one atomic max into mx[slot % MX_SLOTS]
// (non-negative floats order like their bit patterns; spreading the blocks
// over MX_SLOTS words keeps the atomics from queueing on one address).  Every
// thread of the block must call it; wbuf holds one float per wave.
__device__ __forceinline__ void gather_max(unsigned *mx, float m, float *wbuf, int slot) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = absmax(m, __shfl_xor(m, off));
  const int t = threadIdx.x + blockDim.x * threadIdx.y;
  const int nw = (blockDim.x * blockDim.y) >> 6;
  if ((t & 63) == 0) wbuf[t >> 6] = m;
  __syncthreads();
  if (t == 0) {
    for (int i = 1; i < nw; ++i) m = absmax(m, wbuf[i]);
    atomicMax(mx + (slot % MX_SLOTS), __float_as_uint(m));
  }
}


// ---------------------------------------------------------------------------
// Cell products, FP32 vectors (same algorithm as k_cell_gemm):
//   BF16 = false: cell matrices FP32, v_mfma_f32_16x16x4f32, 32 k-steps
//   BF16 = true:  cell matrices BF16 (row-major), the gathered tile is converted
//                 to BF16 in LDS (stored column-major so that a lane's 8
//                 consecutive k values are contiguous), v_mfma_f32_16x16x32_bf16,
//                 4 k-steps
// ---------------------------------------------------------------------------
// One cell per workgroup of 512 threads; slot picks the max-gathering word.
template <bool BF16, int NSB>
__device__ __forceinline__ void cell_gemm_lp_body(
    const void *__restrict__ Hv, const int32_t *__restrict__ dofp,
    const uint8_t *__restrict__ flagp, const int cell,
    const float *__restrict__ X, int64_t ldx, float *__restrict__ Y, int64_t ldy, int N,
    const CellFinishF &f, int slot) {
  // column tiles of NSB (1 or 2) 16-column MFMA blocks: two fill a 128-byte
  // line per gathered row, one keeps the registers low (the faster choice
  // depends on the form and the problem; the results are the same)
  static_assert(NSB == 1 || NSB == 2, "one or two column blocks per tile");
  constexpr int NT = NSB * CELL_NT;
  constexpr int LDX = NT + 16;               // FP32 tile, row-major [k][col]
  constexpr int LDT = NPAD + 8;              // BF16 tile, column-major [col][k]
  constexpr int PF = NPAD * NT / 512;
  constexpr int RPP = 512 / NT;
  __shared__ float xs[BF16 ? 1 : NPAD * LDX];
  __shared__ __bf16 xt[BF16 ? NT * LDT : 8];
  __shared__ float xk_tile[BF16 ? NPAD * NT : 1];   // FP32 copy for the finishing step
  __shared__ int32_t sdof[NPAD];
  __shared__ uint8_t sflag[NPAD];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  if (tid < NPAD) {
    sdof[tid] = dofp[(int64_t)cell * NPAD + tid];
    sflag[tid] = flagp[(int64_t)cell * NPAD + tid];
  }
  float a32[BF16 ? 1 : 32];
  bf8 a16[BF16 ? 4 : 1];
  if constexpr (BF16) {
    const __bf16 *Hc = (const __bf16 *)Hv + (int64_t)cell * NPAD * NPAD;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      a16[ks] = *(const bf8 *)(Hc + (16 * w + li) * NPAD + 32 * ks + 8 * kq);
  } else {
    const float *Hc = (const float *)Hv + (int64_t)cell * NPAD * NPAD;
#pragma unroll
    for (int ks = 0; ks < 32; ++ks) a32[ks] = Hc[(4 * ks + kq) * NPAD + 16 * w + li];
  }
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
  float pf[PF];
  auto gather = [&](int c) {
    const int col = min(c + gj, N - 1);
#pragma unroll
    for (int p = 0; p < PF; ++p) pf[p] = X[gd[p] * ldx + col];
  };
  gather(0);
  const bool finish = f.Out != nullptr;
  float fc1 = f.c1, fc2 = f.c2, fc3 = f.c3;
  if (f.mult) {
    const float al = f.mult[0], be = f.mult[1];
    fc1 *= al; fc2 *= al; fc3 *= be;
  }
  float omax = 0.f;
  int od[4];
  bool ofirst[4], ofin[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * w + 4 * kq + r;
    od[r] = sdof[row];
    ofirst[r] = (sflag[row] & CELL_FIRST) != 0;
    ofin[r] = finish && od[r] >= 0 && (sflag[row] & CELL_FINISH) != 0;
  }
  // the scaled inverse mass of the finishing rows, read once
  float dv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) dv[r] = ofin[r] ? fc1 * (float)f.dinv[od[r]] : 0.f;

  // old Y (and Yp of finishing rows) of a tile's two column blocks, loaded
  // one tile ahead into one of two register sets
  auto load_y = [&](float (&yo)[NSB][4], float (&yp)[NSB][4], int c) {
#pragma unroll
    for (int sb = 0; sb < NSB; ++sb) {
      const int col = c + 16 * sb + li;
      const bool cv = col < N;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        yo[sb][r] = (od[r] >= 0 && !ofirst[r] && cv) ? Y[(int64_t)od[r] * ldy + col] : 0.f;
        yp[sb][r] = (ofin[r] && f.Yp && cv) ? f.Yp[(int64_t)od[r] * f.ldyp + col] : 0.f;
      }
    }
  };
  // A tile's results are stored during the next tile, after that tile's
  // gathered rows have gone to LDS (pending global stores make the wave wait
  // for all of its memory operations before the fill).
  float out[NSB][4];
  auto store_out = [&](int c0) {
#pragma unroll
    for (int sb = 0; sb < NSB; ++sb) {
      const int col = c0 + 16 * sb + li;
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (od[r] < 0) continue;
        if (ofin[r])
          f.Out[(int64_t)od[r] * f.ldo + col] = out[sb][r];
        else
          Y[(int64_t)od[r] * ldy + col] = out[sb][r];
      }
    }
  };
  auto tile = [&](float (&yo)[NSB][4], float (&yp)[NSB][4], float (&yo2)[NSB][4],
                  float (&yp2)[NSB][4], int c0) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int row = gr + p * RPP;
      const float v = (gok[p] && c0 + gj < N) ? pf[p] : 0.f;
      if constexpr (BF16) {
        xt[gj * LDT + row] = (__bf16)v;
        xk_tile[row * NT + gj] = v;
      } else {
        xs[row * LDX + gj] = v;
      }
    }
    if (c0 > 0) store_out(c0 - NT);
    __syncthreads();
    const int c1 = c0 + NT;
    if (c1 < N) {
      gather(c1);
      load_y(yo2, yp2, c1);
    }
    f4 acc[NSB];
#pragma unroll
    for (int sb = 0; sb < NSB; ++sb) {
      acc[sb] = f4zero();
      if (c0 + 16 * sb >= N) break;            // block beyond the last column (uniform)
      if constexpr (BF16) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          acc[sb] = mfma_bf16(a16[ks], *(const bf8 *)(xt + (16 * sb + li) * LDT + 32 * ks + 8 * kq),
                              acc[sb]);
      } else {
#pragma unroll
        for (int ks = 0; ks < 32; ++ks)
          acc[sb] = mfma_f32(a32[ks], xs[(4 * ks + kq) * LDX + 16 * sb + li], acc[sb]);
      }
    }
#pragma unroll
    for (int sb = 0; sb < NSB; ++sb) {
      const bool cv = c0 + 16 * sb + li < N;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = acc[sb][r] + yo[sb][r];
        const int row = 16 * w + 4 * kq + r;
        float xk;
        if constexpr (BF16) xk = xk_tile[row * NT + 16 * sb + li];
        else xk = xs[row * LDX + 16 * sb + li];
        // explicit fused steps: the rounding is the same in every tile shape
        const float o = fmaf(fc3, yp[sb][r], fmaf(fc2, xk, dv[r] * v));
        out[sb][r] = ofin[r] ? o : v;
        if (ofin[r] && cv) omax = absmax(omax, o);
      }
    }
    __syncthreads();
  };
  float ya[NSB][4], pa[NSB][4], yb[NSB][4], pb[NSB][4];
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
  if (f.mx) gather_max(f.mx, omax, (float *)sdof, slot);   // sdof is free after the tile loop
}

// ---------------------------------------------------------------------------
// Coupling partials, FP32 (as k_enr_part; FP32 blocks HT, MT).
// ---------------------------------------------------------------------------
// One enriched cell per workgroup of 512 threads; the blocks are read once per
// call (cells with more than B 16-row blocks take several passes over the
// gathered rows).  8 waves split between B output row blocks and KP = 8 / B
// parts of the 128 local nodes (B = 4: k halves; B = 2: quarters; B = 1:
// eighths), each wave holding the A fragments of both terms for its k part in
// registers; the parts are added through LDS in k-part order.  B is chosen
// per cell from its number of row blocks by the map `bmap` (2 bits per
// bucket of 1, 2, 3, >= 4 row blocks: 0 -> B = 1, 1 -> 2, 2 -> 4), which the
// autotuner sets.  The gathered rows of a tile are loaded one tile ahead into
// registers.
__device__ __forceinline__ int cpl_b(int bmap, int nmb) {
  const int q = nmb < 4 ? nmb - 1 : 3;
  return 1 << ((bmap >> (2 * q)) & 3);
}

template <int B>
__device__ __forceinline__ void enr_part_f32_impl(
    const float *__restrict__ ht, const float *__restrict__ mt, int nap, int nmb, int na,
    int64_t k0, const int (&gd)[4], const float (&gsc)[4], const float *__restrict__ X,
    int64_t ldx, float cH, const float *__restrict__ R, int64_t ldr, float cM,
    float *__restrict__ P, int64_t ldp, int N, float *xs, float *rsm, float *xch) {
  constexpr int PT = 16, LDX = PT + 1, PF = 4, RPP = 32;
  constexpr int KP = 8 / B, KS = NPAD / KP, NKS = KS / 4;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int wb = w % B, h = w / B;
  const int gj = tid % PT, gr = tid / PT;
  for (int g = 0; B * g < nmb; ++g) {
    const int mb = B * g + wb;
    const bool act = mb < nmb;
    float aH[NKS], aM[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int64_t off = (int64_t)(KS * h + 4 * ks + kq) * nap + 16 * mb + li;
      aH[ks] = (act && ht) ? ht[off] : 0.f;
      aM[ks] = (act && mt) ? mt[off] : 0.f;
    }
    // the gathered rows of the next tile, loaded during this tile's MFMAs;
    // the loads are unconditional (row and column clamped) and their values
    // untouched until the LDS store (masking and R scaling there).  A tile's
    // partial sums are stored during the next tile, after its LDS fill.
    float qx[PF], qr[PF], out[4];
    auto gather = [&](int c) {
      const int col = min(c + gj, N - 1);
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int64_t row = gd[p] >= 0 ? gd[p] : 0;
        if (X) qx[p] = X[row * ldx + col];
        if (R) qr[p] = R[row * ldr + col];
      }
    };
    auto store_out = [&](int c0) {
      if (act && h == 0 && c0 + li < N) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int orow = 16 * mb + 4 * kq + r;
          if (orow < na) P[(k0 + orow) * ldp + c0 + li] = out[r];
        }
      }
    };
    gather(0);
    for (int c0 = 0; c0 < N; c0 += PT) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const bool v = gd[p] >= 0 && c0 + gj < N;
        xs[(gr + p * RPP) * LDX + gj] = (X && v) ? qx[p] : 0.f;
        rsm[(gr + p * RPP) * LDX + gj] = (R && v) ? qr[p] * gsc[p] : 0.f;
      }
      if (c0 > 0) store_out(c0 - PT);
      __syncthreads();
      if (c0 + PT < N) gather(c0 + PT);
      f4 acc = f4zero();
      if (act) {
        f4 accH = f4zero(), accM = f4zero();
        if (ht) {
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks)
            accH = mfma_f32(aH[ks], xs[(KS * h + 4 * ks + kq) * LDX + li], accH);
        }
        if (mt) {
#pragma unroll
          for (int ks = 0; ks < NKS; ++ks)
            accM = mfma_f32(aM[ks], rsm[(KS * h + 4 * ks + kq) * LDX + li], accM);
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
          float v = acc[r];
#pragma unroll
          for (int q = 1; q < KP; ++q) v += xch[(((q - 1) * B + wb) * 4 + r) * 64 + lane];
          out[r] = v;
        }
      }
    }
    store_out(PT * ((N - 1) / PT));
    __syncthreads();
  }
}

__device__ __forceinline__ void enr_part_f32_body(
    const float *__restrict__ HT, const float *__restrict__ MT,
    const int64_t *__restrict__ toff, const int32_t *__restrict__ tld,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ dofp,
    const int cell, const float *__restrict__ X, int64_t ldx, float cH,
    const float *__restrict__ R, int64_t ldr, const double *__restrict__ rs, float cM,
    float *__restrict__ P, int64_t ldp, int N, int bmap) {
  constexpr int PT = 16, LDX = PT + 1, PF = 4, RPP = 32;
  __shared__ float xs[NPAD * LDX];
  __shared__ float rsm[NPAD * LDX];
  __shared__ float xch[7 * 4 * 64];          // partial sums of k parts 1..KP-1
  const int tid = threadIdx.x;
  const int gr = tid / PT;
  int gd[PF];
  float gsc[PF];
#pragma unroll
  for (int p = 0; p < PF; ++p) {
    gd[p] = dofp[(int64_t)cell * NPAD + gr + p * RPP];
    gsc[p] = (rs && gd[p] >= 0) ? (float)rs[gd[p]] : 1.f;
  }
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  const int nap = tld[cell];
  const int nmb = nap >> 4;
  const float *ht = X ? HT + toff[cell] : nullptr;
  const float *mt = R ? MT + toff[cell] : nullptr;
  if (nmb == 0) return;
  const int B = cpl_b(bmap, nmb);
  if (B == 4)
    enr_part_f32_impl<4>(ht, mt, nap, nmb, na, k0, gd, gsc, X, ldx, cH, R, ldr, cM, P, ldp, N, xs,
                         rsm, xch);
  else if (B == 2)
    enr_part_f32_impl<2>(ht, mt, nap, nmb, na, k0, gd, gsc, X, ldx, cH, R, ldr, cM, P, ldp, N, xs,
                         rsm, xch);
  else
    enr_part_f32_impl<1>(ht, mt, nap, nmb, na, k0, gd, gsc, X, ldx, cH, R, ldr, cM, P, ldp, N, xs,
                         rsm, xch);
}

// ---------------------------------------------------------------------------
// Transposed coupling products, FP32 (as k_enr_q): U rows FP32, V rows FP64
// (the Schur-solve output), products in FP32.
// ---------------------------------------------------------------------------
// One enriched cell per workgroup of 256 threads; its rows of Q start at
// 128 * qblock (the cell's position in the enriched-cell list).  The
// enrichment functions are taken in chunks of 64: wave w keeps the A fragments
// of rows 32w .. 32w+32 of both blocks for the chunk in registers while the
// column tiles stream by; chunks after the first add into Q.
__device__ __forceinline__ void enr_q_f32_body(
    const float *__restrict__ Hec, const float *__restrict__ Mec,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ eidx,
    const int cell, const int qblock, const float *__restrict__ U, int64_t ldu, float cU,
    const double *__restrict__ V, int64_t ldv, float cV, float *__restrict__ Q, int64_t ldq,
    int N) {
  constexpr int PT = 16, LDZ = 16, KC = 64, KS = KC / 4;
  constexpr int GV = KC * PT / 256;
  __shared__ float zu[KC * LDZ];
  __shared__ float zv[KC * LDZ];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  float *qb = Q + ((int64_t)qblock * NPAD) * ldq;
  const int gj = tid % PT, gk = tid / PT;
  for (int kc = 0; kc < na; kc += KC) {
    float aH0[KS], aH1[KS], aM0[KS], aM1[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = kc + 4 * ks + kq;
      const bool v = k < na;
      const float *hr = Hec + (k0 + (v ? k : 0)) * NPAD + 32 * w;
      const float *mr = Mec + (k0 + (v ? k : 0)) * NPAD + 32 * w;
      aH0[ks] = (U && v) ? hr[li] : 0.f;
      aH1[ks] = (U && v) ? hr[16 + li] : 0.f;
      aM0[ks] = (V && v) ? mr[li] : 0.f;
      aM1[ks] = (V && v) ? mr[16 + li] : 0.f;
    }
    int64_t gal[GV];
    bool gv[GV];
#pragma unroll
    for (int p = 0; p < GV; ++p) {
      const int k = kc + gk + 16 * p;
      gv[p] = k < na;
      gal[p] = gv[p] ? eidx[k0 + k] : 0;
    }
    // the next tile's gathered rows, loaded during this tile's MFMAs
    // (unconditional loads, column clamped; scaled and masked at the LDS
    // store); a tile's Q values are stored during the next tile, after its
    // LDS fill
    float pu[GV], o0[4], o1[4];
    double pv[GV];
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
        float *q = qb + c0 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          q[(int64_t)(32 * w + 4 * kq + r) * ldq] = o0[r];
          q[(int64_t)(32 * w + 16 + 4 * kq + r) * ldq] = o1[r];
        }
      }
    };
    gather(0);
    for (int c0 = 0; c0 < N; c0 += PT) {
      const int ncol = min(PT, N - c0);
#pragma unroll
      for (int p = 0; p < GV; ++p) {
        const bool v = gv[p] && c0 + gj < N;
        zu[(gk + 16 * p) * LDZ + gj] = (U && v) ? cU * pu[p] : 0.f;
        zv[(gk + 16 * p) * LDZ + gj] = (V && v) ? cV * (float)pv[p] : 0.f;
      }
      if (c0 > 0) store_q(c0 - PT);
      __syncthreads();
      if (c0 + PT < N) gather(c0 + PT);
      // chunks after the first add into Q: its old values, loaded before the
      // products so that their latency overlaps them
      float qo0[4], qo1[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ld = kc > 0 && li < ncol;
        const float *q = qb + c0 + li;
        qo0[r] = ld ? q[(int64_t)(32 * w + 4 * kq + r) * ldq] : 0.f;
        qo1[r] = ld ? q[(int64_t)(32 * w + 16 + 4 * kq + r) * ldq] : 0.f;
      }
      f4 acc0 = f4zero(), acc1 = f4zero();
      if (U) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const float b = zu[(4 * ks + kq) * LDZ + li];
          acc0 = mfma_f32(aH0[ks], b, acc0);
          acc1 = mfma_f32(aH1[ks], b, acc1);
        }
      }
      if (V) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const float b = zv[(4 * ks + kq) * LDZ + li];
          acc0 = mfma_f32(aM0[ks], b, acc0);
          acc1 = mfma_f32(aM1[ks], b, acc1);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        o0[r] = acc0[r] + qo0[r];
        o1[r] = acc1[r] + qo1[r];
      }
      __syncthreads();
    }
    store_q(PT * ((N - 1) / PT));
  }
  if (na == 0) {
    for (int c0 = 0; c0 < N; c0 += PT)
      for (int idx = tid; idx < NPAD * PT; idx += 256) {
        const int a = idx / PT, j = idx % PT;
        if (c0 + j < N) qb[(int64_t)a * ldq + c0 + j] = 0.f;
      }
  }
}

// ---------------------------------------------------------------------------
// Enrichment rows from FP32 partials, accumulated in FP64:
//   out[al,:] = sum_{k in list(al)} P[k,:] + sum_be Dn[al,be] Zd[be,:]     (Zd FP32)
// ---------------------------------------------------------------------------
// The sums of one element are split into 4 contiguous quarters of the
// partial list and of the dense product, each summed in index order from zero
// and combined as ((q0 + q1) + q2) + q3: the batched form adds the quarters
// one after the other, the single-problem kernel gives each quarter a wave;
// the bits are the same.  Loads are issued 8 at a time before their adds.
__device__ __forceinline__ void enr_reduce_f32_quarter(
    int n_e, const int64_t *__restrict__ aptr, const int32_t *__restrict__ alist,
    const float *__restrict__ P, int64_t ldp, const double *__restrict__ Dn,
    const float *__restrict__ Zd, int64_t ldzd, int al, int col, int w, double &sp, double &sd) {
  constexpr int U = 8;
  sp = 0.0;
  sd = 0.0;
  const int64_t a0 = aptr[al], len = aptr[al + 1] - a0;
  const int64_t q0 = a0 + (len * w) / 4, q1 = a0 + (len * (w + 1)) / 4;
  int64_t k = q0;
  for (; k + U <= q1; k += U) {
    float t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = P[(int64_t)alist[k + u] * ldp + col];
#pragma unroll
    for (int u = 0; u < U; ++u) sp += (double)t[u];
  }
  for (; k < q1; ++k) sp += (double)P[(int64_t)alist[k] * ldp + col];
  const double *drow = Dn + (int64_t)al * n_e;
  const int b0 = (n_e * w) / 4, b1 = (n_e * (w + 1)) / 4;
  int be = b0;
  for (; be + U <= b1; be += U) {
    float t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = Zd[(int64_t)(be + u) * ldzd + col];
#pragma unroll
    for (int u = 0; u < U; ++u) sd += drow[be + u] * (double)t[u];
  }
  for (; be < b1; ++be) sd += drow[be] * (double)Zd[(int64_t)be * ldzd + col];
}

__device__ __forceinline__ void enr_reduce_f32_elem(
    int n_e, const int64_t *__restrict__ aptr, const int32_t *__restrict__ alist,
    const float *__restrict__ P, int64_t ldp, const double *__restrict__ Dn,
    const float *__restrict__ Zd, int64_t ldzd, double *__restrict__ out, int64_t ldo, int al,
    int col) {
  double sp[4], sd[4];
#pragma unroll
  for (int w = 0; w < 4; ++w)
    enr_reduce_f32_quarter(n_e, aptr, alist, P, ldp, Dn, Zd, ldzd, al, col, w, sp[w], sd[w]);
  out[(int64_t)al * ldo + col] =
      (((sp[0] + sp[1]) + sp[2]) + sp[3]) + (((sd[0] + sd[1]) + sd[2]) + sd[3]);
}

// ---------------------------------------------------------------------------
// Epilogue, FP32 blocks (as k_epilogue): rows = listed classical rows, then the
// enrichment rows (Ee FP64, converted).
// ---------------------------------------------------------------------------
// Block of 64 x 4 threads; this block takes rows t = 4 b0 + threadIdx.y,
// t += 4 bstride.  When every block's rows start on 16-byte boundaries a lane
// takes 4 adjacent columns with vector loads, and a DOF's (at most 8) buffer
// rows are loaded before any of them is added, so the loads of an element are
// all in flight together; the arithmetic of an element (sum order included)
// is the same in both mappings.
constexpr int EPI_F32_QMAX = 8;
__device__ __forceinline__ void epilogue_f32_body(const EpiArgsF &g, int64_t b0, int64_t bstride,
                                                  int slot) {
  const int64_t ncls = g.rows ? g.nrows : g.n_h;
  const int64_t nt = ncls + g.n_e;
  float gc1 = g.c1, gc2 = g.c2, gc3 = g.c3;
  if (g.mult) {
    const float al = g.mult[0], be = g.mult[1];
    gc1 *= al; gc2 *= al; gc3 *= be;
  }
  auto a16 = [](const void *ptr, int64_t ld, int64_t elems) {
    return ptr == nullptr || (((uintptr_t)ptr & 15) == 0 && (ld * elems) % 16 == 0);
  };
  const bool vec = a16(g.R, g.ldr, 4) && a16(g.Q, g.ldq, 4) && a16(g.Ee, g.lde, 8) &&
                   a16(g.Yk, g.ldyk, 4) && a16(g.Yp, g.ldyp, 4) && a16(g.Out, g.ldo, 4);
  float omax = 0.f;
  for (int64_t t = b0 * 4 + threadIdx.y; t < nt; t += bstride * 4) {
    const bool cls = t < ncls;
    const int64_t i = cls ? (g.rows ? (int64_t)g.rows[t] : t) : g.n_h + (t - ncls);
    float dr = 1.f;
    int p0 = 0, p1 = 0;
    if (cls) {
      if (g.dinv) dr = (float)g.dinv[i];
      if (g.qptr) { p0 = g.qptr[i]; p1 = g.qptr[i + 1]; }
    }
    const int nq = p1 - p0;
    // one element, the loads of its buffer rows given
    auto elem = [&](float r, const float *qv, double e, float yk, float yp) {
      float v;
      if (cls) {
        float s = r;
        for (int u = 0; u < nq; ++u) s += qv[u];
        v = dr * s;
      } else {
        v = (float)e;
      }
      v *= gc1;
      if (g.Yk) v += gc2 * yk;
      if (g.Yp) v += gc3 * yp;
      omax = absmax(omax, v);
      return v;
    };
    if (vec && nq <= EPI_F32_QMAX) {
      int64_t qo[EPI_F32_QMAX];
#pragma unroll
      for (int u = 0; u < EPI_F32_QMAX; ++u) qo[u] = u < nq ? (int64_t)g.qidx[p0 + u] * g.ldq : 0;
      for (int j = 4 * threadIdx.x; j < g.N; j += 256) {
        if (j + 3 < g.N) {
          const float4 r = cls ? *reinterpret_cast<const float4 *>(g.R + i * g.ldr + j)
                               : float4{0.f, 0.f, 0.f, 0.f};
          double2 e0{0.0, 0.0}, e1{0.0, 0.0};
          if (!cls) {
            e0 = *reinterpret_cast<const double2 *>(g.Ee + (i - g.n_h) * g.lde + j);
            e1 = *reinterpret_cast<const double2 *>(g.Ee + (i - g.n_h) * g.lde + j + 2);
          }
          float4 q[EPI_F32_QMAX];
#pragma unroll
          for (int u = 0; u < EPI_F32_QMAX; ++u)
            q[u] = u < nq ? *reinterpret_cast<const float4 *>(g.Q + qo[u] + j)
                          : float4{0.f, 0.f, 0.f, 0.f};
          const float4 yk = g.Yk ? *reinterpret_cast<const float4 *>(g.Yk + i * g.ldyk + j)
                                 : float4{0.f, 0.f, 0.f, 0.f};
          const float4 yp = g.Yp ? *reinterpret_cast<const float4 *>(g.Yp + i * g.ldyp + j)
                                 : float4{0.f, 0.f, 0.f, 0.f};
          float qv[EPI_F32_QMAX];
          float4 o;
#pragma unroll
          for (int u = 0; u < EPI_F32_QMAX; ++u) qv[u] = q[u].x;
          o.x = elem(r.x, qv, e0.x, yk.x, yp.x);
#pragma unroll
          for (int u = 0; u < EPI_F32_QMAX; ++u) qv[u] = q[u].y;
          o.y = elem(r.y, qv, e0.y, yk.y, yp.y);
#pragma unroll
          for (int u = 0; u < EPI_F32_QMAX; ++u) qv[u] = q[u].z;
          o.z = elem(r.z, qv, e1.x, yk.z, yp.z);
#pragma unroll
          for (int u = 0; u < EPI_F32_QMAX; ++u) qv[u] = q[u].w;
          o.w = elem(r.w, qv, e1.y, yk.w, yp.w);
          *reinterpret_cast<float4 *>(g.Out + i * g.ldo + j) = o;
        } else {
          for (int jj = j; jj < g.N; ++jj) {
            float qv[EPI_F32_QMAX];
#pragma unroll
            for (int u = 0; u < EPI_F32_QMAX; ++u) qv[u] = u < nq ? g.Q[qo[u] + jj] : 0.f;
            g.Out[i * g.ldo + jj] =
                elem(cls ? g.R[i * g.ldr + jj] : 0.f, qv, cls ? 0.0 : g.Ee[(i - g.n_h) * g.lde + jj],
                     g.Yk ? g.Yk[i * g.ldyk + jj] : 0.f, g.Yp ? g.Yp[i * g.ldyp + jj] : 0.f);
          }
        }
      }
    } else {
      for (int j = threadIdx.x; j < g.N; j += 64) {
        float v;
        if (cls) {
          float s = g.R[i * g.ldr + j];
          for (int p = p0; p < p1; ++p) s += g.Q[(int64_t)g.qidx[p] * g.ldq + j];
          v = dr * s;
        } else {
          v = (float)g.Ee[(i - g.n_h) * g.lde + j];
        }
        v *= gc1;
        if (g.Yk) v += gc2 * g.Yk[i * g.ldyk + j];
        if (g.Yp) v += gc3 * g.Yp[i * g.ldyp + j];
        g.Out[i * g.ldo + j] = v;
        omax = absmax(omax, v);
      }
    }
  }
  if (g.mx) {
    // every thread of the block reaches this point (the row loop has no early exit)
    __shared__ float wbuf[4];
    gather_max(g.mx, omax, wbuf, slot);
  }
}

// ---------------------------------------------------------------------------
// Scaled recurrence bookkeeping
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lp_input_body(int64_t rows, int N, const double *__restrict__ X,
                                              int64_t ldx, float *__restrict__ Z, int64_t ldz,
                                              unsigned *__restrict__ mx0, int64_t b0,
                                              int64_t bstride, int slot) {
  float m = 0.f;
  for (int64_t i = b0 * 4 + threadIdx.y; i < rows; i += bstride * 4)
    for (int j = threadIdx.x; j < N; j += 64) {
      const float z = (float)X[i * ldx + j];
      Z[i * ldz + j] = z;
      m = absmax(m, z);
    }
  __shared__ float wbuf[4];
  gather_max(mx0, m, wbuf, slot);
}

// Scale of step k (which forms Z_k+1 from Z_k, Z_k-1): the exponent of
// max|Y_k+1| is predicted from the last two iterates, E_k+1 ~ 2 E_k - E_k-1
// (Chebyshev growth per step settles to a constant), and s_k+1 is set to it,
// so that max|Z_k+1| stays near 1; at most 60 binades from s_k.  Step 0 is not
// scaled.  A zero or non-finite maximum keeps the previous scale.
__device__ __forceinline__ void lp_scale_body(int k, const unsigned *__restrict__ mx,
                                              int32_t *__restrict__ sexp, float *__restrict__ mult) {
  if (k == 0) {
    sexp[0] = 0;
    sexp[1] = 0;
    mult[0] = 1.f;
    mult[1] = 1.f;
    return;
  }
  const int sk = sexp[k], sp = sexp[k - 1];
  unsigned uk = 0u, up = 0u;
  for (int i = 0; i < MX_SLOTS; ++i) {
    uk = max(uk, mx[k * MX_SLOTS + i]);
    up = max(up, mx[(k - 1) * MX_SLOTS + i]);
  }
  const float mk = __uint_as_float(uk), mp = __uint_as_float(up);
  int sn = sk;
  if (mk > 0.f && mp > 0.f && isfinite(mk) && isfinite(mp)) {
    int ek, ep;
    (void)frexpf(mk, &ek);
    (void)frexpf(mp, &ep);
    const int pred = 2 * (ek + sk) - (ep + sp);
    sn = min(max(pred, sk - 60), sk + 60);
  }
  sexp[k + 1] = sn;
  mult[2 * k] = ldexpf(1.f, sk - sn);
  mult[2 * k + 1] = ldexpf(1.f, sp - sn);
}

__device__ __forceinline__ void lp_output_body(int64_t rows, int N, const float *__restrict__ Z,
                                               int64_t ldz, const int32_t *__restrict__ sexp_m,
                                               double *__restrict__ Y, int64_t ldy, int64_t b0,
                                               int64_t bstride) {
  const int sm = *sexp_m;
  for (int64_t i = b0 * 4 + threadIdx.y; i < rows; i += bstride * 4)
    for (int j = threadIdx.x; j < N; j += 64) Y[i * ldy + j] = ldexp((double)Z[i * ldz + j], sm);
}

}  // namespace lowp
}  // namespace cf
