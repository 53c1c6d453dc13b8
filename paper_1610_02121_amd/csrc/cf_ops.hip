// Elemental operator kernels: classical cell products on FP64 MFMA, the
// enriched-classical coupling products, enrichment-row reductions and the
// Chebyshev recurrence epilogue (Sec. IV.D, Sec. V).
//
// MFMA fragment layout of v_mfma_f64_16x16x4f64 (wave of 64 lanes):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element r holds D[4 * r + l / 16][l % 16]
#include "cf_kernels.h"

namespace cf {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 d4zero() { d4 z = {0.0, 0.0, 0.0, 0.0}; return z; }

// ---------------------------------------------------------------------------
// Classical cell products.  One workgroup (4 waves) per cell of the colour.
// The cell matrix (padded to 128 x 128, symmetric) lives in registers as MFMA
// A fragments for the whole call: wave w owns output rows [32w, 32w+32).  The
// block is walked in column tiles of CT: the gathered X rows of the cell are
// staged in LDS (Dirichlet and padding rows are zero), multiplied, and the
// result is written (first touch) or added to the cell's DOF rows of Y.  No
// two cells of one colour share a DOF, so the read-modify-write is race free.
// ---------------------------------------------------------------------------
template <int NTILE>
__global__ __launch_bounds__(256, 2) void k_cell_gemm(
    const double *__restrict__ Hp, const int32_t *__restrict__ dofp,
    const uint8_t *__restrict__ firstp, const int32_t *__restrict__ cells,
    const double *__restrict__ X, int64_t ldx, double *__restrict__ Y, int64_t ldy, int N) {
  constexpr int LDX = NTILE + 16;   // row stride: 16-double pad keeps B-fragment reads conflict free
  __shared__ double xs[NPAD * LDX];
  __shared__ int32_t sdof[NPAD];
  __shared__ uint8_t sfirst[NPAD];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int cell = cells[blockIdx.x];
  if (tid < NPAD) {
    sdof[tid] = dofp[(int64_t)cell * NPAD + tid];
    sfirst[tid] = firstp[(int64_t)cell * NPAD + tid];
  }
  const double *Hc = Hp + (int64_t)cell * NPAD * NPAD;
  // A[i][k] = H[i][k] = H[k][i]: lane reads H[4ks + kq][row] (contiguous in row)
  double a0[32], a1[32];
#pragma unroll
  for (int ks = 0; ks < 32; ++ks) {
    a0[ks] = Hc[(4 * ks + kq) * NPAD + 32 * w + li];
    a1[ks] = Hc[(4 * ks + kq) * NPAD + 32 * w + 16 + li];
  }
  __syncthreads();

  for (int c0 = 0; c0 < N; c0 += NTILE) {
    const int ncol = min(NTILE, N - c0);
    for (int idx = tid; idx < NPAD * NTILE; idx += 256) {
      const int r = idx / NTILE, j = idx % NTILE;
      const int d = sdof[r];
      double v = 0.0;
      if (d >= 0 && j < ncol) v = X[(int64_t)d * ldx + c0 + j];
      xs[r * LDX + j] = v;
    }
    __syncthreads();
    const int ncb = (ncol + 15) >> 4;
    d4 acc0[NTILE / 16], acc1[NTILE / 16];
#pragma unroll
    for (int cb = 0; cb < NTILE / 16; ++cb) { acc0[cb] = d4zero(); acc1[cb] = d4zero(); }
#pragma unroll
    for (int ks = 0; ks < 32; ++ks) {
#pragma unroll
      for (int cb = 0; cb < NTILE / 16; ++cb) {
        if (cb < ncb) {
          const double b = xs[(4 * ks + kq) * LDX + 16 * cb + li];
          acc0[cb] = mfma_f64(a0[ks], b, acc0[cb]);
          acc1[cb] = mfma_f64(a1[ks], b, acc1[cb]);
        }
      }
    }
#pragma unroll
    for (int cb = 0; cb < NTILE / 16; ++cb) {
      const int col = 16 * cb + li;
      if (cb < ncb && col < ncol) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row0 = 32 * w + kq + 4 * r;
          const int d0 = sdof[row0];
          if (d0 >= 0) {
            double *p = Y + (int64_t)d0 * ldy + c0 + col;
            *p = sfirst[row0] ? acc0[cb][r] : *p + acc0[cb][r];
          }
          const int row1 = row0 + 16;
          const int d1 = sdof[row1];
          if (d1 >= 0) {
            double *p = Y + (int64_t)d1 * ldy + c0 + col;
            *p = sfirst[row1] ? acc1[cb][r] : *p + acc1[cb][r];
          }
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_cell_gemm(hipStream_t s, const double *Hp, const int32_t *dofp,
                            const uint8_t *firstp, const int32_t *cells, int ncells,
                            const double *X, int64_t ldx, double *Y, int64_t ldy, int N) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  // narrow blocks (a single vector in the Lanczos run) use a 16-column instance
  if (N <= 16)
    hipLaunchKernelGGL(k_cell_gemm<16>, dim3(ncells), dim3(256), 0, s, Hp, dofp, firstp, cells, X,
                       ldx, Y, ldy, N);
  else
    hipLaunchKernelGGL(k_cell_gemm<CT>, dim3(ncells), dim3(256), 0, s, Hp, dofp, firstp, cells, X,
                       ldx, Y, ldy, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transposed coupling for enriched cells of one colour (grid: cells x column
// tiles): Y[dof(e,a)] += sign * sum_k B[k0+k][a] Z[idx[k0+k]].  The gathered
// enrichment rows sit in LDS (dynamic size: kmax rounded to 4 rows).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_enr_T(
    const double *__restrict__ Bp, const int64_t *__restrict__ eptr,
    const int32_t *__restrict__ eidx, const int32_t *__restrict__ dofp,
    const int32_t *__restrict__ cells, const double *__restrict__ Z, int64_t ldz,
    double *__restrict__ Y, int64_t ldy, int N, double sign) {
  extern __shared__ double zs[];
  constexpr int LDZ = CT + 16;
  __shared__ int32_t sdof[NPAD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int cell = cells[blockIdx.x];
  const int c0 = blockIdx.y * CT;
  const int ncol = min(CT, N - c0);
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  const int K4 = (na + 3) & ~3;
  if (tid < NPAD) sdof[tid] = dofp[(int64_t)cell * NPAD + tid];
  for (int idx = tid; idx < K4 * CT; idx += 256) {
    const int k = idx / CT, j = idx % CT;
    double v = 0.0;
    if (k < na && j < ncol) v = Z[(int64_t)eidx[k0 + k] * ldz + c0 + j];
    zs[k * LDZ + j] = v;
  }
  __syncthreads();
  d4 acc0[CT / 16], acc1[CT / 16];
#pragma unroll
  for (int cb = 0; cb < CT / 16; ++cb) { acc0[cb] = d4zero(); acc1[cb] = d4zero(); }
  for (int ks = 0; ks < K4 / 4; ++ks) {
    const int k = 4 * ks + kq;
    double a0 = 0.0, a1 = 0.0;
    if (k < na) {
      const double *brow = Bp + (k0 + k) * NPAD + 32 * w;
      a0 = brow[li];
      a1 = brow[16 + li];
    }
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) {
      const double b = zs[k * LDZ + 16 * cb + li];
      acc0[cb] = mfma_f64(a0, b, acc0[cb]);
      acc1[cb] = mfma_f64(a1, b, acc1[cb]);
    }
  }
#pragma unroll
  for (int cb = 0; cb < CT / 16; ++cb) {
    const int col = 16 * cb + li;
    if (col < ncol) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row0 = 32 * w + kq + 4 * r;
        const int d0 = sdof[row0];
        if (d0 >= 0) Y[(int64_t)d0 * ldy + c0 + col] += sign * acc0[cb][r];
        const int d1 = sdof[row0 + 16];
        if (d1 >= 0) Y[(int64_t)d1 * ldy + c0 + col] += sign * acc1[cb][r];
      }
    }
  }
}

hipError_t launch_enr_T(hipStream_t s, const double *Bp, const int64_t *eptr,
                        const int32_t *eidx, const int32_t *dofp, const int32_t *cells,
                        int ncells, int kmax, const double *Z, int64_t ldz, double *Y,
                        int64_t ldy, int N, double sign) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  const size_t shm = (size_t)((kmax + 3) & ~3) * (CT + 16) * sizeof(double);
  static size_t shm_set = 0;
  if (shm > 65536 && shm > shm_set) {
    hipError_t e = hipFuncSetAttribute((const void *)k_enr_T,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    shm_set = shm;
  }
  dim3 grid(ncells, (N + CT - 1) / CT);
  hipLaunchKernelGGL(k_enr_T, grid, dim3(256), shm, s, Bp, eptr, eidx, dofp, cells, Z, ldz, Y,
                     ldy, N, sign);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Coupling partials for enriched cells (grid: cells x column tiles):
//   P[k0+k] = sum_a B[k0+k][a] * scale(dof) * Zc[dof(e,a)]
// Each wave takes 16-row blocks of the cell's enrichment rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_enr_N(
    const double *__restrict__ Bp, const int64_t *__restrict__ eptr,
    const int32_t *__restrict__ dofp, const int32_t *__restrict__ cells,
    const double *__restrict__ Zc, int64_t ldz, const double *__restrict__ dscale,
    double *__restrict__ P, int64_t ldp, int N) {
  constexpr int LDX = CT + 16;
  __shared__ double xs[NPAD * LDX];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, kq = lane >> 4;
  const int cell = cells[blockIdx.x];
  const int c0 = blockIdx.y * CT;
  const int ncol = min(CT, N - c0);
  for (int idx = tid; idx < NPAD * CT; idx += 256) {
    const int r = idx / CT, j = idx % CT;
    const int d = dofp[(int64_t)cell * NPAD + r];
    double v = 0.0;
    if (d >= 0 && j < ncol) {
      v = Zc[(int64_t)d * ldz + c0 + j];
      if (dscale) v *= dscale[d];
    }
    xs[r * LDX + j] = v;
  }
  __syncthreads();
  const int64_t k0 = eptr[cell];
  const int na = (int)(eptr[cell + 1] - k0);
  const int nmb = (na + 15) >> 4;
  for (int mb = w; mb < nmb; mb += 4) {
    d4 acc[CT / 16];
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) acc[cb] = d4zero();
    const int arow = 16 * mb + li;
    const bool valid = arow < na;
    const double *brow = Bp + (k0 + (valid ? arow : 0)) * NPAD;
#pragma unroll 8
    for (int ks = 0; ks < 32; ++ks) {
      const double a = valid ? brow[4 * ks + kq] : 0.0;
#pragma unroll
      for (int cb = 0; cb < CT / 16; ++cb) {
        const double b = xs[(4 * ks + kq) * LDX + 16 * cb + li];
        acc[cb] = mfma_f64(a, b, acc[cb]);
      }
    }
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) {
      const int col = 16 * cb + li;
      if (col < ncol) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int orow = 16 * mb + kq + 4 * r;
          if (orow < na) P[(k0 + orow) * ldp + c0 + col] = acc[cb][r];
        }
      }
    }
  }
}

hipError_t launch_enr_N(hipStream_t s, const double *Bp, const int64_t *eptr,
                        const int32_t *dofp, const int32_t *cells, int ncells,
                        const double *Zc, int64_t ldz, const double *dscale, double *P,
                        int64_t ldp, int N) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  dim3 grid(ncells, (N + CT - 1) / CT);
  hipLaunchKernelGGL(k_enr_N, grid, dim3(256), 0, s, Bp, eptr, dofp, cells, Zc, ldz, dscale, P,
                     ldp, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Enrichment rows (grid: column tiles of 64 x n_e): fixed-order segmented sum
// of the per-cell partials, plus an optional dense n_e x n_e product and an
// optional scaled extra term.  Deterministic: no atomics.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_enr_reduce(
    int n_e, const int64_t *__restrict__ aptr, const int32_t *__restrict__ alist,
    const double *__restrict__ P, int64_t ldp, double s_p, const double *__restrict__ R0,
    int64_t ldr0, double s_r, const double *__restrict__ Dn, const double *__restrict__ Zd,
    int64_t ldzd, double *__restrict__ out, int64_t ldo, int N) {
  const int col = blockIdx.x * 64 + threadIdx.x;
  const int al = blockIdx.y;
  if (col >= N) return;
  double acc = 0.0;
  if (P) {
    double sp = 0.0;
    for (int64_t k = aptr[al]; k < aptr[al + 1]; ++k) sp += P[(int64_t)alist[k] * ldp + col];
    acc = s_p * sp;
  }
  if (R0) acc += s_r * R0[(int64_t)al * ldr0 + col];
  if (Dn) {
    const double *drow = Dn + (int64_t)al * n_e;
    double sd = 0.0;
    for (int be = 0; be < n_e; ++be) sd += drow[be] * Zd[(int64_t)be * ldzd + col];
    acc += sd;
  }
  out[(int64_t)al * ldo + col] = acc;
}

hipError_t launch_enr_reduce(hipStream_t s, int n_e, const int64_t *aptr, const int32_t *alist,
                             const double *P, int64_t ldp, double s_p, const double *R0,
                             int64_t ldr0, double s_r, const double *Dn, const double *Zd,
                             int64_t ldzd, double *out, int64_t ldo, int N) {
  if (n_e <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + 63) / 64, n_e);
  hipLaunchKernelGGL(k_enr_reduce, grid, dim3(64), 0, s, n_e, aptr, alist, P, ldp, s_p, R0, ldr0,
                     s_r, Dn, Zd, ldzd, out, ldo, N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Recurrence epilogue: block (64 columns x 4 rows), grid-stride over rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_epilogue(
    int64_t n_h, int64_t n_e, const double *__restrict__ dinv, const double *__restrict__ R,
    int64_t ldr, const double *__restrict__ Ze, int64_t ldze, double c1,
    const double *__restrict__ Yk, int64_t ldyk, double c2, const double *Yp, int64_t ldyp,
    double c3, double *Out, int64_t ldo, int N) {
  const int64_t n = n_h + n_e;
  for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.y; i < n; i += (int64_t)gridDim.x * 4) {
    const bool cls = i < n_h;
    const double di = cls ? dinv[i] : 0.0;
    for (int j = threadIdx.x; j < N; j += 64) {
      double v = cls ? di * R[i * ldr + j] : Ze[(i - n_h) * ldze + j];
      v *= c1;
      if (Yk) v += c2 * Yk[i * ldyk + j];
      if (Yp) v += c3 * Yp[i * ldyp + j];
      Out[i * ldo + j] = v;
    }
  }
}

hipError_t launch_epilogue(hipStream_t s, int64_t n_h, int64_t n_e, const double *dinv,
                           const double *R, int64_t ldr, const double *Ze, int64_t ldze,
                           double c1, const double *Yk, int64_t ldyk, double c2,
                           const double *Yp, int64_t ldyp, double c3, double *Out,
                           int64_t ldo, int N) {
  const int64_t n = n_h + n_e;
  if (n <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_epilogue, dim3((unsigned)blocks), dim3(64, 4), 0, s, n_h, n_e, dinv, R, ldr,
                     Ze, ldze, c1, Yk, ldyk, c2, Yp, ldyp, c3, Out, ldo, N);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_diag_scale(int64_t rows, const double *__restrict__ d,
                                                    const double *X, int64_t ldx, double *Out,
                                                    int64_t ldo, int N) {
  for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.y; i < rows; i += (int64_t)gridDim.x * 4) {
    const double di = d[i];
    for (int j = threadIdx.x; j < N; j += 64) Out[i * ldo + j] = di * X[i * ldx + j];
  }
}

hipError_t launch_diag_scale(hipStream_t s, int64_t rows, const double *d, const double *X,
                             int64_t ldx, double *Out, int64_t ldo, int N) {
  if (rows <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (rows + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_diag_scale, dim3((unsigned)blocks), dim3(64, 4), 0, s, rows, d, X, ldx, Out,
                     ldo, N);
  return hipGetLastError();
}

}  // namespace cf
