// Element blocks of the cells outside every enrichment support (Sec. III.B,
// Eq. HBlocks): H_cc_e = K + B^T diag(w .* V_e) B, where K (the kinetic
// block 1/2 int grad N_a . grad N_b) is the same for every cell of the
// uniform mesh, B [nq][npc] holds the shape-function values at the cell's
// Gauss points (reference coordinates, the same for every cell), w the
// weights with the Jacobian, and V_e the potential at the cell's points.
// The quadrature sum is a dense contraction over the nq points: it runs on
// FP64 MFMA, one workgroup per cell.
#include "cf_kernels.h"

namespace cf {

typedef double d4 __attribute__((ext_vector_type(4)));

// The 36 16 x 16 tiles (ti <= tj) of the upper triangle of the 128 x 128
// block, dealt to the 4 waves of a workgroup round robin (9 each).
__host__ __device__ constexpr int up_ti(int t) {
  int i = 0;
  while (t >= 8 - i) { t -= 8 - i; ++i; }
  return i;
}
__host__ __device__ constexpr int up_tj(int t) {
  int i = 0;
  while (t >= 8 - i) { t -= 8 - i; ++i; }
  return i + t;
}

template <int T>
__device__ __forceinline__ d4 tile_mfma(const double (&val)[8], double s, d4 acc) {
  constexpr int ti = up_ti(T), tj = up_tj(T);
  return __builtin_amdgcn_mfma_f64_16x16x4f64(val[ti] * s, val[tj], acc, 0, 0, 0);
}

// Exact symmetry: the value at (row <= col) is written at (row, col) and (col, row).
template <int T>
__device__ __forceinline__ void tile_store(const d4 &acc, const double *__restrict__ K,
                                           double *__restrict__ He) {
  constexpr int ti = up_ti(T), tj = up_tj(T);
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lr = 4 * r + kq;
    if (ti == tj && lr > li) continue;
    const int row = 16 * ti + lr, col = 16 * tj + li;
    const double v = K[row * NPAD + col] + acc[r];
    He[row * NPAD + col] = v;
    if (row != col) He[col * NPAD + row] = v;
  }
}

// One wave's 9 tiles (W, W + 4, ..., W + 32).  v_mfma_f64_16x16x4f64 takes
// A[l % 16][l / 16], B[l / 16][l % 16] and returns D element r of lane l at
// D[4 r + l / 16][l % 16].  Here A[i][k] = B_tab[q0 + k][16 ti + i] s[q0 + k]
// and B[k][j] = B_tab[q0 + k][16 tj + j]: both operands come from the lane's
// table values val[t] = B_tab[q0 + l / 16][16 t + l % 16].
template <int W>
__device__ __forceinline__ void assemble_wave(const double *__restrict__ Btab,
                                              const double *__restrict__ wq,
                                              const double *__restrict__ Ve, int nq, int nq4,
                                              const double *__restrict__ K,
                                              double *__restrict__ He) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, kq = lane >> 4;
  d4 acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
  for (int q0 = 0; q0 < nq4; q0 += 4) {
    const int q = q0 + kq;
    const double s = q < nq ? wq[q] * Ve[q] : 0.0;
    double val[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) val[t] = Btab[(int64_t)q * NPAD + 16 * t + li];
    acc[0] = tile_mfma<W + 0>(val, s, acc[0]);
    acc[1] = tile_mfma<W + 4>(val, s, acc[1]);
    acc[2] = tile_mfma<W + 8>(val, s, acc[2]);
    acc[3] = tile_mfma<W + 12>(val, s, acc[3]);
    acc[4] = tile_mfma<W + 16>(val, s, acc[4]);
    acc[5] = tile_mfma<W + 20>(val, s, acc[5]);
    acc[6] = tile_mfma<W + 24>(val, s, acc[6]);
    acc[7] = tile_mfma<W + 28>(val, s, acc[7]);
    acc[8] = tile_mfma<W + 32>(val, s, acc[8]);
  }
  tile_store<W + 0>(acc[0], K, He);
  tile_store<W + 4>(acc[1], K, He);
  tile_store<W + 8>(acc[2], K, He);
  tile_store<W + 12>(acc[3], K, He);
  tile_store<W + 16>(acc[4], K, He);
  tile_store<W + 20>(acc[5], K, He);
  tile_store<W + 24>(acc[6], K, He);
  tile_store<W + 28>(acc[7], K, He);
  tile_store<W + 32>(acc[8], K, He);
}

__global__ __launch_bounds__(256) void k_assemble_cells(const double *__restrict__ Btab,
                                                        const double *__restrict__ wq,
                                                        const double *__restrict__ K,
                                                        const int *__restrict__ cells, int ncells,
                                                        const double *__restrict__ V, int64_t ldv,
                                                        int nq, double *__restrict__ Hp) {
  const int ci = blockIdx.x;
  if (ci >= ncells) return;
  const double *Ve = V + (int64_t)ci * ldv;
  double *He = Hp + (int64_t)cells[ci] * NPAD * NPAD;
  const int nq4 = (nq + 3) & ~3;
  switch (threadIdx.x >> 6) {
    case 0: assemble_wave<0>(Btab, wq, Ve, nq, nq4, K, He); break;
    case 1: assemble_wave<1>(Btab, wq, Ve, nq, nq4, K, He); break;
    case 2: assemble_wave<2>(Btab, wq, Ve, nq, nq4, K, He); break;
    default: assemble_wave<3>(Btab, wq, Ve, nq, nq4, K, He); break;
  }
}

hipError_t launch_assemble_cells(hipStream_t s, const double *Btab, const double *wq,
                                 const double *K, const int *cells, int ncells, const double *V,
                                 int64_t ldv, int nq, double *Hp) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble_cells, dim3((unsigned)ncells), dim3(256), 0, s, Btab, wq, K, cells,
                     ncells, V, ldv, nq, Hp);
  return hipGetLastError();
}

}  // namespace cf
