// Small fully connected network for the learned filter bounds: n_in inputs,
// `depth` hidden layers of `width` units with GELU, n_out linear outputs; FP32
// forward, backward (mean squared error) and Adam, each a hand-written kernel.
// Sizes are tiny (width 128, batches of a few hundred), so every kernel gives
// one output element to one thread and sums in a fixed order: results are
// deterministic.
//
// Parameter layout (flat FP32): for layer l = 0..depth, W_l [out_l][in_l]
// row-major, then b_l [out_l]; in_0 = n_in, out_l = width (l < depth),
// out_depth = n_out.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "chebfilter.h"

namespace {

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * kInvSqrt2)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.f + erff(x * kInvSqrt2)) + x * kInvSqrt2Pi * expf(-0.5f * x * x);
}

// Z[s][o] = b[o] + sum_i A[s][i] W[o][i];  Aout = gelu(Z) or Z
__global__ __launch_bounds__(256) void k_dense_fwd(int B, int in, int out, const float *__restrict__ A,
                                                   const float *__restrict__ W,
                                                   const float *__restrict__ b, float *__restrict__ Z,
                                                   float *__restrict__ Aout, int act) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= B * out) return;
  const int s = idx / out, o = idx % out;
  float acc = b[o];
  const float *a = A + (int64_t)s * in, *w = W + (int64_t)o * in;
  for (int i = 0; i < in; ++i) acc = fmaf(a[i], w[i], acc);
  Z[idx] = acc;
  Aout[idx] = act ? gelu(acc) : acc;
}

// Mean squared error over B x n: loss = sum (Y - T)^2 / (B n), dY = 2 (Y - T) / (B n).
// One block; partial sums in a fixed tree.
__global__ __launch_bounds__(256) void k_mse(int total, const float *__restrict__ Y,
                                             const float *__restrict__ T, float *__restrict__ dY,
                                             float *__restrict__ loss) {
  __shared__ float red[256];
  const float inv = 1.f / (float)total;
  float acc = 0.f;
  for (int i = threadIdx.x; i < total; i += 256) {
    const float d = Y[i] - T[i];
    dY[i] = 2.f * d * inv;
    acc = fmaf(d, d, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * inv;
}

// dZ = dA * gelu'(Z)  (or dA for a linear layer)
__global__ __launch_bounds__(256) void k_dact(int n, const float *__restrict__ dA,
                                              const float *__restrict__ Z, float *__restrict__ dZ,
                                              int act) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dZ[i] = act ? dA[i] * gelu_grad(Z[i]) : dA[i];
}

// dW[o][i] = sum_s dZ[s][o] A[s][i];  db[o] = sum_s dZ[s][o]  (thread i == 0 of row o)
__global__ __launch_bounds__(256) void k_dense_bwd_w(int B, int in, int out,
                                                     const float *__restrict__ dZ,
                                                     const float *__restrict__ A,
                                                     float *__restrict__ dW, float *__restrict__ db) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= out * in) return;
  const int o = idx / in, i = idx % in;
  float acc = 0.f;
  for (int s = 0; s < B; ++s) acc = fmaf(dZ[(int64_t)s * out + o], A[(int64_t)s * in + i], acc);
  dW[idx] = acc;
  if (i == 0) {
    float ab = 0.f;
    for (int s = 0; s < B; ++s) ab += dZ[(int64_t)s * out + o];
    db[o] = ab;
  }
}

// dA[s][i] = sum_o dZ[s][o] W[o][i]
__global__ __launch_bounds__(256) void k_dense_bwd_x(int B, int in, int out,
                                                     const float *__restrict__ dZ,
                                                     const float *__restrict__ W,
                                                     float *__restrict__ dA) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= B * in) return;
  const int s = idx / in, i = idx % in;
  float acc = 0.f;
  for (int o = 0; o < out; ++o) acc = fmaf(dZ[(int64_t)s * out + o], W[(int64_t)o * in + i], acc);
  dA[idx] = acc;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m / bc1) / (sqrt(v / bc2) + eps), bc = 1 - beta^t.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float *__restrict__ p,
                                              const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct cf_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_in = 0, width = 0, depth = 0, n_out = 0, max_batch = 0;
  std::vector<int> din, dout;
  std::vector<int64_t> woff, boff;
  int64_t nparams = 0;
  float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
  std::vector<float *> Z, A;     // per layer pre-activation / activation (A[0] = input copy)
  float *dA = nullptr, *dB = nullptr, *dZ = nullptr, *Tbuf = nullptr, *loss = nullptr;
  int64_t step = 0;
  std::vector<double> norm;      // in_mean, in_std, out_mean, out_std (empty = identity)
  std::string err;
  std::vector<void *> allocs;
};

namespace {

thread_local std::string g_mlp_error;

cf_status merr(cf_mlp *m, cf_status st, const std::string &msg) {
  if (m) m->err = msg; else g_mlp_error = msg;
  return st;
}

#define MHIP(m, call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return merr(m, CF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

cf_status malloc_f(cf_mlp *m, float **p, int64_t n) {
  void *q = nullptr;
  if (hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return merr(m, CF_ENOMEM, "mlp: hipMalloc failed");
  }
  m->allocs.push_back(q);
  *p = (float *)q;
  return CF_OK;
}

void free_mlp(cf_mlp *m) {
  if (!m) return;
  for (void *q : m->allocs) (void)hipFree(q);
  delete m;
}

cf_status forward(cf_mlp *m, const float *X, int B) {
  MHIP(m, hipMemcpyAsync(m->A[0], X, (size_t)B * m->n_in * sizeof(float), hipMemcpyDeviceToDevice,
                         m->stream));
  const int L = m->depth + 1;
  for (int l = 0; l < L; ++l) {
    const int in = m->din[l], out = m->dout[l];
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks_for((int64_t)B * out)), dim3(256), 0, m->stream, B,
                       in, out, m->A[l], m->params + m->woff[l], m->params + m->boff[l], m->Z[l],
                       m->A[l + 1], l < m->depth ? 1 : 0);
    MHIP(m, hipGetLastError());
  }
  return CF_OK;
}

}  // namespace

extern "C" {

cf_status chebfilter_mlp_create(int32_t device, void *stream, int32_t n_in, int32_t width,
                                int32_t depth, int32_t n_out, int32_t max_batch, cf_mlp **out) {
  if (!out) return merr(nullptr, CF_EINVAL, "mlp_create: null output pointer");
  *out = nullptr;
  if (n_in < 1 || width < 1 || depth < 1 || n_out < 1 || max_batch < 1 || n_in > 4096 ||
      width > 4096 || depth > 16 || n_out > 4096)
    return merr(nullptr, CF_EINVAL, "mlp_create: bad sizes");
  cf_mlp *m = new (std::nothrow) cf_mlp();
  if (!m) return merr(nullptr, CF_ENOMEM, "mlp_create: host allocation failed");
  m->device = device;
  m->stream = (hipStream_t)stream;
  m->n_in = n_in; m->width = width; m->depth = depth; m->n_out = n_out; m->max_batch = max_batch;
  if (hipSetDevice(device) != hipSuccess) { free_mlp(m); return merr(nullptr, CF_EDEVICE, "mlp_create: hipSetDevice failed"); }
  const int L = depth + 1;
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int in = l == 0 ? n_in : width, o = l < depth ? width : n_out;
    m->din.push_back(in);
    m->dout.push_back(o);
    m->woff.push_back(off);
    off += (int64_t)in * o;
    m->boff.push_back(off);
    off += o;
  }
  m->nparams = off;
  cf_status st = CF_OK;
  auto A = [&](float **p, int64_t n) { if (st == CF_OK) st = malloc_f(m, p, n); };
  A(&m->params, off); A(&m->grads, off); A(&m->am, off); A(&m->av, off);
  const int wmax = std::max(std::max(n_in, width), n_out);
  m->Z.assign(L, nullptr);
  m->A.assign(L + 1, nullptr);
  for (int l = 0; l < L; ++l) A(&m->Z[l], (int64_t)max_batch * m->dout[l]);
  A(&m->A[0], (int64_t)max_batch * n_in);
  for (int l = 0; l < L; ++l) A(&m->A[l + 1], (int64_t)max_batch * m->dout[l]);
  A(&m->dA, (int64_t)max_batch * wmax); A(&m->dB, (int64_t)max_batch * wmax);
  A(&m->dZ, (int64_t)max_batch * wmax); A(&m->Tbuf, (int64_t)max_batch * n_out); A(&m->loss, 4);
  if (st != CF_OK) { g_mlp_error = m->err; free_mlp(m); return st; }
  if (hipMemset(m->params, 0, off * sizeof(float)) != hipSuccess ||
      hipMemset(m->am, 0, off * sizeof(float)) != hipSuccess ||
      hipMemset(m->av, 0, off * sizeof(float)) != hipSuccess) {
    free_mlp(m);
    return merr(nullptr, CF_EDEVICE, "mlp_create: hipMemset failed");
  }
  *out = m;
  return CF_OK;
}

cf_status chebfilter_mlp_destroy(cf_mlp *m) {
  if (!m) return CF_OK;
  (void)hipSetDevice(m->device);
  (void)hipStreamSynchronize(m->stream);
  free_mlp(m);
  return CF_OK;
}

const char *chebfilter_mlp_last_error(const cf_mlp *m) { return m ? m->err.c_str() : g_mlp_error.c_str(); }

cf_status chebfilter_mlp_sizes(const cf_mlp *m, int64_t *nparams) {
  if (!m) return CF_EINVAL;
  if (nparams) *nparams = m->nparams;
  return CF_OK;
}

cf_status chebfilter_mlp_set_params(cf_mlp *m, const float *host, int32_t reset_adam) {
  if (!m || !host) return CF_EINVAL;
  MHIP(m, hipSetDevice(m->device));
  MHIP(m, hipMemcpyAsync(m->params, host, m->nparams * sizeof(float), hipMemcpyHostToDevice, m->stream));
  if (reset_adam) {
    std::vector<float> z(m->nparams, 0.f);
    MHIP(m, hipMemcpyAsync(m->am, z.data(), m->nparams * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MHIP(m, hipMemcpyAsync(m->av, z.data(), m->nparams * sizeof(float), hipMemcpyHostToDevice, m->stream));
    m->step = 0;
  }
  MHIP(m, hipStreamSynchronize(m->stream));
  return CF_OK;
}

cf_status chebfilter_mlp_get_params(cf_mlp *m, float *host) {
  if (!m || !host) return CF_EINVAL;
  MHIP(m, hipSetDevice(m->device));
  MHIP(m, hipMemcpyAsync(host, m->params, m->nparams * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MHIP(m, hipStreamSynchronize(m->stream));
  return CF_OK;
}

cf_status chebfilter_mlp_forward(cf_mlp *m, const float *X, int32_t B, float *Y) {
  if (!m || !X || !Y) return CF_EINVAL;
  if (B < 1 || B > m->max_batch) return merr(m, CF_EINVAL, "mlp_forward: B out of [1, max_batch]");
  MHIP(m, hipSetDevice(m->device));
  {
    cf_status st = forward(m, X, B);
    if (st != CF_OK) return st;
  }
  MHIP(m, hipMemcpyAsync(Y, m->A[m->depth + 1], (size_t)B * m->n_out * sizeof(float),
                         hipMemcpyDeviceToDevice, m->stream));
  return CF_OK;
}

cf_status chebfilter_mlp_loss_grad(cf_mlp *m, const float *X, const float *T, int32_t B,
                                   float *loss_host, float *grad_host) {
  if (!m || !X || !T) return CF_EINVAL;
  if (B < 1 || B > m->max_batch) return merr(m, CF_EINVAL, "mlp_loss_grad: B out of [1, max_batch]");
  MHIP(m, hipSetDevice(m->device));
  {
    cf_status st = forward(m, X, B);
    if (st != CF_OK) return st;
  }
  const int L = m->depth + 1;
  const int total = B * m->n_out;
  // dY into dA
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, m->stream, total, m->A[L], T, m->dA, m->loss);
  MHIP(m, hipGetLastError());
  float *dAcur = m->dA, *dAnext = m->dB;
  for (int l = L - 1; l >= 0; --l) {
    const int in = m->din[l], out = m->dout[l];
    hipLaunchKernelGGL(k_dact, dim3(blocks_for((int64_t)B * out)), dim3(256), 0, m->stream, B * out,
                       dAcur, m->Z[l], m->dZ, l < m->depth ? 1 : 0);
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks_for((int64_t)out * in)), dim3(256), 0, m->stream, B,
                       in, out, m->dZ, m->A[l], m->grads + m->woff[l], m->grads + m->boff[l]);
    if (l > 0)
      hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks_for((int64_t)B * in)), dim3(256), 0, m->stream, B,
                         in, out, m->dZ, m->params + m->woff[l], dAnext);
    MHIP(m, hipGetLastError());
    std::swap(dAcur, dAnext);
  }
  if (loss_host)
    MHIP(m, hipMemcpyAsync(loss_host, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  if (grad_host)
    MHIP(m, hipMemcpyAsync(grad_host, m->grads, m->nparams * sizeof(float), hipMemcpyDeviceToHost,
                           m->stream));
  MHIP(m, hipStreamSynchronize(m->stream));
  return CF_OK;
}

cf_status chebfilter_mlp_adam_step(cf_mlp *m, float lr, float beta1, float beta2, float eps) {
  if (!m) return CF_EINVAL;
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return merr(m, CF_EINVAL, "mlp_adam_step: bad hyper-parameters");
  MHIP(m, hipSetDevice(m->device));
  m->step += 1;
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)m->step));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)m->step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(m->nparams)), dim3(256), 0, m->stream, m->nparams,
                     m->params, m->grads, m->am, m->av, lr, beta1, beta2, eps, bc1, bc2);
  MHIP(m, hipGetLastError());
  return CF_OK;
}

cf_status chebfilter_mlp_set_normalization(cf_mlp *m, const double *in_mean, const double *in_std,
                                           const double *out_mean, const double *out_std) {
  if (!m || !in_mean || !in_std || !out_mean || !out_std) return CF_EINVAL;
  std::vector<double> nv;
  for (int i = 0; i < m->n_in; ++i) nv.push_back(in_mean[i]);
  for (int i = 0; i < m->n_in; ++i) {
    if (!(in_std[i] > 0.0)) return merr(m, CF_EINVAL, "mlp_set_normalization: std must be > 0");
    nv.push_back(in_std[i]);
  }
  for (int i = 0; i < m->n_out; ++i) nv.push_back(out_mean[i]);
  for (int i = 0; i < m->n_out; ++i) {
    if (!(out_std[i] > 0.0)) return merr(m, CF_EINVAL, "mlp_set_normalization: std must be > 0");
    nv.push_back(out_std[i]);
  }
  m->norm = nv;
  return CF_OK;
}

// Normalisation fitted to a corpus (count samples, row-major): per column the
// mean and the standard deviation; a standard deviation below 1e-12 (1 + |mean|)
// (a constant column) is replaced by 1.
cf_status chebfilter_mlp_fit_normalization(cf_mlp *m, const double *inputs, const double *targets,
                                           int64_t count) {
  if (!m || !inputs || !targets || count < 1) return CF_EINVAL;
  auto stats = [count](const double *x, int cols, std::vector<double> &mean, std::vector<double> &sd) {
    mean.assign(cols, 0.0);
    sd.assign(cols, 0.0);
    for (int64_t r = 0; r < count; ++r)
      for (int j = 0; j < cols; ++j) mean[j] += x[r * cols + j];
    for (int j = 0; j < cols; ++j) mean[j] /= (double)count;
    for (int64_t r = 0; r < count; ++r)
      for (int j = 0; j < cols; ++j) {
        const double d = x[r * cols + j] - mean[j];
        sd[j] += d * d;
      }
    for (int j = 0; j < cols; ++j) {
      sd[j] = std::sqrt(sd[j] / (double)count);
      if (!(sd[j] > 1e-12 * (1.0 + std::fabs(mean[j])))) sd[j] = 1.0;
    }
  };
  std::vector<double> im, is, om, os;
  stats(inputs, m->n_in, im, is);
  stats(targets, m->n_out, om, os);
  return chebfilter_mlp_set_normalization(m, im.data(), is.data(), om.data(), os.data());
}

// Normalised copies (FP32) of raw inputs (which = 0) or targets (which = 1),
// [count][n_in or n_out], with the network's current normalisation.
cf_status chebfilter_mlp_normalize(cf_mlp *m, int32_t which, const double *x, int64_t count,
                                   float *out) {
  if (!m || !x || !out || count < 0 || (which != 0 && which != 1)) return CF_EINVAL;
  if (m->norm.empty()) return merr(m, CF_EINVAL, "mlp_normalize: normalisation not set");
  const int cols = which == 0 ? m->n_in : m->n_out;
  const double *mean = m->norm.data() + (which == 0 ? 0 : 2 * m->n_in);
  const double *sd = mean + cols;
  for (int64_t r = 0; r < count; ++r)
    for (int j = 0; j < cols; ++j) out[r * cols + j] = (float)((x[r * cols + j] - mean[j]) / sd[j]);
  return CF_OK;
}

extern "C++" cf_status cf_mlp_predict_raw(cf_mlp *m, const double *x_raw, double *y_raw);

// Raw outputs of raw inputs, sample by sample through the normalisation.
cf_status chebfilter_mlp_predict(cf_mlp *m, const double *x_raw, int64_t count, double *y_raw) {
  if (!m || !x_raw || !y_raw || count < 0) return CF_EINVAL;
  for (int64_t r = 0; r < count; ++r) {
    cf_status st = cf_mlp_predict_raw(m, x_raw + r * m->n_in, y_raw + r * m->n_out);
    if (st != CF_OK) return st;
  }
  return CF_OK;
}

}  // extern "C"

// Used by chebfilter_bounds_predict (cf_api.hip): raw inputs -> raw outputs
// through the normalisation; synchronises.
cf_status cf_mlp_predict_raw(cf_mlp *m, const double *x_raw, double *y_raw) {
  if (m->norm.empty()) return merr(m, CF_EINVAL, "bounds_predict: normalisation not set");
  std::vector<float> x(m->n_in), y(m->n_out);
  const double *im = m->norm.data(), *is = im + m->n_in, *om = is + m->n_in, *os = om + m->n_out;
  for (int i = 0; i < m->n_in; ++i) x[i] = (float)((x_raw[i] - im[i]) / is[i]);
  MHIP(m, hipSetDevice(m->device));
  MHIP(m, hipMemcpyAsync(m->dB, x.data(), m->n_in * sizeof(float), hipMemcpyHostToDevice, m->stream));
  {
    cf_status st = forward(m, m->dB, 1);
    if (st != CF_OK) return st;
  }
  MHIP(m, hipMemcpyAsync(y.data(), m->A[m->depth + 1], m->n_out * sizeof(float),
                         hipMemcpyDeviceToHost, m->stream));
  MHIP(m, hipStreamSynchronize(m->stream));
  for (int i = 0; i < m->n_out; ++i) y_raw[i] = om[i] + os[i] * (double)y[i];
  return CF_OK;
}

int cf_mlp_n_in(const cf_mlp *m) { return m->n_in; }
int cf_mlp_n_out(const cf_mlp *m) { return m->n_out; }
const char *cf_mlp_err(const cf_mlp *m) { return m->err.c_str(); }
