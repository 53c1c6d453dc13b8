// Reduced-precision operator kernels for the filter's matrix products (FP32
// vectors; cell products on FP32 MFMA, or BF16 inputs with FP32 accumulation;
// coupling products on FP32 MFMA).  The enrichment reductions accumulate in
// FP64 and the Schur-complement solve stays FP64 (cf_ops.hip).  Structure,
// flags and data layouts follow the FP64 kernels of cf_ops.hip; the kernel
// bodies are in cf_lowp_body.h.
#include "cf_lowp_body.h"

namespace cf {

using namespace lowp;

template <bool BF16, int NSB>
__global__ __launch_bounds__(512, 2) void k_cell_gemm_lp(
    const void *__restrict__ Hv, const int32_t *__restrict__ dofp,
    const uint8_t *__restrict__ flagp, const int32_t *__restrict__ cells,
    const float *__restrict__ X, int64_t ldx, float *__restrict__ Y, int64_t ldy, int N,
    const CellFinishF f) {
  cell_gemm_lp_body<BF16, NSB>(Hv, dofp, flagp, cells[blockIdx.x], X, ldx, Y, ldy, N, f,
                               blockIdx.x);
}

hipError_t launch_cell_gemm_lp(hipStream_t s, bool bf16, int nsb, const void *Hv,
                               const int32_t *dofp, const uint8_t *flagp, const int32_t *cells,
                               int ncells, const float *X, int64_t ldx, float *Y, int64_t ldy,
                               int N, const CellFinishF &f) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  if (nsb != 1 && nsb != 2) return hipErrorInvalidValue;
  auto kern = bf16 ? (nsb == 2 ? k_cell_gemm_lp<true, 2> : k_cell_gemm_lp<true, 1>)
                   : (nsb == 2 ? k_cell_gemm_lp<false, 2> : k_cell_gemm_lp<false, 1>);
  hipLaunchKernelGGL(kern, dim3(ncells), dim3(512), 0, s, Hv, dofp, flagp, cells, X, ldx, Y, ldy,
                     N, f);
  return hipGetLastError();
}

__global__ __launch_bounds__(512, 2) void k_enr_part_f32(
    const float *__restrict__ HT, const float *__restrict__ MT,
    const int64_t *__restrict__ toff, const int32_t *__restrict__ tld,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ dofp,
    const int32_t *__restrict__ cells, const float *__restrict__ X, int64_t ldx, float cH,
    const float *__restrict__ R, int64_t ldr, const double *__restrict__ rs, float cM,
    float *__restrict__ P, int64_t ldp, int N, int bmap) {
  enr_part_f32_body(HT, MT, toff, tld, eptr, dofp, cells[blockIdx.x], X, ldx, cH, R, ldr, rs, cM, P,
                    ldp, N, bmap);
}

hipError_t launch_enr_part_f32(hipStream_t s, const float *HT, const float *MT,
                               const int64_t *toff, const int32_t *tld, const int64_t *eptr,
                               const int32_t *dofp, const int32_t *cells, int ncells,
                               const float *X, int64_t ldx, float cH, const float *R,
                               int64_t ldr, const double *rs, float cM, float *P, int64_t ldp,
                               int N, int bmap) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_enr_part_f32, dim3(ncells), dim3(512), 0, s, HT, MT, toff, tld, eptr, dofp,
                     cells, X, ldx, cH, R, ldr, rs, cM, P, ldp, N, bmap);
  return hipGetLastError();
}

__global__ __launch_bounds__(256, 2) void k_enr_q_f32(
    const float *__restrict__ Hec, const float *__restrict__ Mec,
    const int64_t *__restrict__ eptr, const int32_t *__restrict__ eidx,
    const int32_t *__restrict__ cells, const int32_t *__restrict__ order,
    const float *__restrict__ U, int64_t ldu, float cU,
    const double *__restrict__ V, int64_t ldv, float cV, float *__restrict__ Q, int64_t ldq,
    int N) {
  const int pos = order ? order[blockIdx.x] : (int)blockIdx.x;   // position in the cell list
  enr_q_f32_body(Hec, Mec, eptr, eidx, cells[pos], pos, U, ldu, cU, V, ldv, cV, Q, ldq, N);
}

hipError_t launch_enr_q_f32(hipStream_t s, const float *Hec, const float *Mec,
                            const int64_t *eptr, const int32_t *eidx, const int32_t *cells,
                            const int32_t *order, int ncells, int kmax, const float *U,
                            int64_t ldu, float cU, const double *V, int64_t ldv, float cV,
                            float *Q, int64_t ldq, int N) {
  if (ncells <= 0 || N <= 0) return hipSuccess;
  (void)kmax;
  hipLaunchKernelGGL(k_enr_q_f32, dim3(ncells), dim3(256), 0, s, Hec, Mec, eptr, eidx, cells, order,
                     U, ldu, cU, V, ldv, cV, Q, ldq, N);
  return hipGetLastError();
}

// One wave per quarter of each element's sums (see enr_reduce_f32_elem),
// combined in quarter order: the same bits as the batched form.
__global__ __launch_bounds__(256) void k_enr_reduce_f32(
    int n_e, const int64_t *__restrict__ aptr, const int32_t *__restrict__ alist,
    const float *__restrict__ P, int64_t ldp, const double *__restrict__ Dn,
    const float *__restrict__ Zd, int64_t ldzd, double *__restrict__ out, int64_t ldo, int N) {
  __shared__ double part[2][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + lane;
  const int al = blockIdx.y;
  double sp = 0.0, sd = 0.0;
  if (col < N)
    enr_reduce_f32_quarter(n_e, aptr, alist, P, ldp, Dn, Zd, ldzd, al, col, w, sp, sd);
  part[0][w][lane] = sp;
  part[1][w][lane] = sd;
  __syncthreads();
  if (w == 0 && col < N)
    out[(int64_t)al * ldo + col] =
        (((part[0][0][lane] + part[0][1][lane]) + part[0][2][lane]) + part[0][3][lane]) +
        (((part[1][0][lane] + part[1][1][lane]) + part[1][2][lane]) + part[1][3][lane]);
}

hipError_t launch_enr_reduce_f32(hipStream_t s, int n_e, const int64_t *aptr,
                                 const int32_t *alist, const float *P, int64_t ldp,
                                 const double *Dn, const float *Zd, int64_t ldzd, double *out,
                                 int64_t ldo, int N) {
  if (n_e <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + 63) / 64, n_e);
  hipLaunchKernelGGL(k_enr_reduce_f32, grid, dim3(256), 0, s, n_e, aptr, alist, P, ldp, Dn, Zd, ldzd,
                     out, ldo, N);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_epilogue_f32(const EpiArgsF g) {
  epilogue_f32_body(g, blockIdx.x, gridDim.x, blockIdx.x);
}

hipError_t launch_epilogue_f32(hipStream_t s, const EpiArgsF &g) {
  const int64_t n = (g.rows ? g.nrows : g.n_h) + g.n_e;
  if (n <= 0 || g.N <= 0) return hipSuccess;
  int64_t blocks = (n + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_epilogue_f32, dim3((unsigned)blocks), dim3(64, 4), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conversions
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_to_f32(int64_t n, const double *__restrict__ x,
                                                float *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    y[i] = (float)x[i];
}
// FP64 -> BF16 with one rounding (to nearest, ties to even) on the FP64 bits:
// the significand is cut to BF16's 8 bits, after which the value is exact in
// FP32 and in BF16 (finite values in BF16's normal range).
__global__ __launch_bounds__(256) void k_to_bf16(int64_t n, const double *__restrict__ x,
                                                 __bf16 *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint64_t b = (uint64_t)__double_as_longlong(x[i]);
    b += ((uint64_t)1 << 44) - 1 + ((b >> 45) & 1);
    b &= ~(((uint64_t)1 << 45) - 1);
    y[i] = (__bf16)(float)__longlong_as_double((long long)b);
  }
}
// Y (type To) [rows][ldy] <- X (type Ti) [rows][ldx], N columns
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_block_convert(int64_t rows, int N, const Ti *__restrict__ X,
                                                       int64_t ldx, To *__restrict__ Y, int64_t ldy) {
  for (int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.y; i < rows; i += (int64_t)gridDim.x * 4)
    for (int j = threadIdx.x; j < N; j += 64) Y[i * ldy + j] = (To)X[i * ldx + j];
}

hipError_t launch_to_f32(hipStream_t s, int64_t n, const double *x, float *y) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}
hipError_t launch_to_bf16(hipStream_t s, int64_t n, const double *x, void *y) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)blocks), dim3(256), 0, s, n, x, (__bf16 *)y);
  return hipGetLastError();
}
hipError_t launch_block_d2f(hipStream_t s, int64_t rows, int N, const double *X, int64_t ldx,
                            float *Y, int64_t ldy) {
  if (rows <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (rows + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_block_convert<double, float>), dim3((unsigned)blocks), dim3(64, 4), 0, s, rows,
                     N, X, ldx, Y, ldy);
  return hipGetLastError();
}
hipError_t launch_block_f2d(hipStream_t s, int64_t rows, int N, const float *X, int64_t ldx,
                            double *Y, int64_t ldy) {
  if (rows <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (rows + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_block_convert<float, double>), dim3((unsigned)blocks), dim3(64, 4), 0, s, rows,
                     N, X, ldx, Y, ldy);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scaled recurrence bookkeeping (bodies in cf_lowp_body.h)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lp_reset(unsigned *__restrict__ mx, int nslots) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nslots; i += gridDim.x * 256) mx[i] = 0u;
}

// Blocks of 64 x 4 threads; rows i = 4 b0 + threadIdx.y, i += 4 bstride.
__global__ __launch_bounds__(256) void k_lp_input(int64_t rows, int N, const double *__restrict__ X,
                                                  int64_t ldx, float *__restrict__ Z, int64_t ldz,
                                                  unsigned *__restrict__ mx0) {
  lp_input_body(rows, N, X, ldx, Z, ldz, mx0, blockIdx.x, gridDim.x, blockIdx.x);
}

__global__ void k_lp_scale(int k, const unsigned *__restrict__ mx, int32_t *__restrict__ sexp,
                           float *__restrict__ mult) {
  if (threadIdx.x == 0 && blockIdx.x == 0) lp_scale_body(k, mx, sexp, mult);
}

__global__ __launch_bounds__(256) void k_lp_output(int64_t rows, int N, const float *__restrict__ Z,
                                                   int64_t ldz, const int32_t *__restrict__ sexp_m,
                                                   double *__restrict__ Y, int64_t ldy) {
  lp_output_body(rows, N, Z, ldz, sexp_m, Y, ldy, blockIdx.x, gridDim.x);
}

hipError_t launch_lp_reset(hipStream_t s, unsigned *mx, int nslots) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lp_reset, dim3((nslots + 255) / 256), dim3(256), 0, s, mx, nslots);
  return hipGetLastError();
}
hipError_t launch_lp_input(hipStream_t s, int64_t rows, int N, const double *X, int64_t ldx,
                           float *Z, int64_t ldz, unsigned *mx0) {
  if (rows <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (rows + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_lp_input, dim3((unsigned)blocks), dim3(64, 4), 0, s, rows, N, X, ldx, Z, ldz,
                     mx0);
  return hipGetLastError();
}
hipError_t launch_lp_scale(hipStream_t s, int k, const unsigned *mx, int32_t *sexp, float *mult) {
  hipLaunchKernelGGL(k_lp_scale, dim3(1), dim3(64), 0, s, k, mx, sexp, mult);
  return hipGetLastError();
}
hipError_t launch_lp_output(hipStream_t s, int64_t rows, int N, const float *Z, int64_t ldz,
                            const int32_t *sexp_m, double *Y, int64_t ldy) {
  if (rows <= 0 || N <= 0) return hipSuccess;
  int64_t blocks = (rows + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_lp_output, dim3((unsigned)blocks), dim3(64, 4), 0, s, rows, N, Z, ldz, sexp_m,
                     Y, ldy);
  return hipGetLastError();
}

}  // namespace cf
