// Online neural synthetic gradients (Sec. III-B/C/E, Alg. 1): per-block
// samples of the two-scale scheme, a fully-connected network of four ReLU
// hidden layers and a linear output, trained by Adam on mean-squared-error
// mini-batches and queried for the synthetic gradient of every block.
//
// Layout: float32 throughout.  A batch of B samples of F features is stored
// sample-major (row r at r * F), i.e. column-major F x B, which is what the
// dense products take.  Layer l's weights are stored row-major out x in
// (column-major in x out), followed by its bias; all layers in one vector.
// The dense products are rocBLAS single-precision GEMMs; everything else
// (sample assembly, bias and ReLU, loss, bias gradients, ReLU masks, Adam)
// is in the kernels below.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <string>

#include "fe_abi.h"
#include "fe_internal.h"

namespace {

constexpr int NL = 5;  // linear layers: 4 hidden + output
constexpr int TPB = 256;

inline int blocks_for(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  return (int)(b < 65535 ? (b < 1 ? 1 : b) : 65535);
}

// corner q of a brick in the local order (x fastest within a face, then z)
__constant__ int c_qx[8] = {0, 1, 1, 0, 0, 1, 1, 0};
__constant__ int c_qy[8] = {0, 0, 1, 1, 0, 0, 1, 1};
__constant__ int c_qz[8] = {0, 0, 0, 0, 1, 1, 1, 1};

struct Blocks {
  int nx, ny, nb, cx, cy, nblk, nin, nout;  // fine grid, block size, coarse grid, sizes
};

// max |x| over n values into *out (one workgroup; the maximum does not
// depend on the order)
__global__ void __launch_bounds__(1024) absmax_kernel(int64_t n, const double* __restrict__ x,
                                                      double* __restrict__ out) {
  __shared__ double part[1024];
  double m = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += 1024) m = fmax(m, fabs(x[t]));
  part[threadIdx.x] = m;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

// Inputs (and with g, targets) of blocks blk0 .. blk0 + n - 1 into rows of X
// (and Y): the block's design variables (x fastest, then y, then z), then
// the 24 coarse displacements of its coarse element over *s_u; targets are
// the block's gradients over *s_g (each computed in float64, then rounded).
// A zero scale leaves the values unscaled.
__global__ void __launch_bounds__(TPB) samples_kernel(Blocks bk, int blk0, int n, const double* __restrict__ z,
                                                      const double* __restrict__ uc, const double* __restrict__ g,
                                                      const double* __restrict__ scales, float* __restrict__ X,
                                                      float* __restrict__ Y) {
  const double s_u = scales[0] > 0.0 ? scales[0] : 1.0;
  const double s_g = (g && scales[1] > 0.0) ? scales[1] : 1.0;
  const int64_t total = (int64_t)n * bk.nin;
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < total; t += (int64_t)gridDim.x * TPB) {
    const int r = (int)(t / bk.nin), f = (int)(t % bk.nin);
    const int blk = blk0 + r;
    const int I = blk % bk.cx, J = (blk / bk.cx) % bk.cy, K = blk / (bk.cx * bk.cy);
    const int nb3 = bk.nb * bk.nb * bk.nb;
    if (f < nb3) {
      const int a = f % bk.nb, b = (f / bk.nb) % bk.nb, c = f / (bk.nb * bk.nb);
      const int64_t e = (bk.nb * I + a) + (int64_t)bk.nx * ((bk.nb * J + b) + (int64_t)bk.ny * (bk.nb * K + c));
      X[t] = (float)z[e];
      if (Y) Y[(int64_t)r * bk.nout + f] = (float)(g[e] / s_g);
    } else {
      const int q = (f - nb3) / 3, d = (f - nb3) % 3;
      const int64_t node = (I + c_qx[q]) + (int64_t)(bk.cx + 1) * ((J + c_qy[q]) + (int64_t)(bk.cy + 1) * (K + c_qz[q]));
      X[t] = (float)(uc[3 * node + d] / s_u);
    }
  }
}

// g of the fine elements of blocks blk0 .. blk0 + n - 1 from the output rows
__global__ void __launch_bounds__(TPB) scatter_kernel(Blocks bk, int blk0, int n, const float* __restrict__ out,
                                                      double* __restrict__ g) {
  const int64_t total = (int64_t)n * bk.nout;
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < total; t += (int64_t)gridDim.x * TPB) {
    const int r = (int)(t / bk.nout), l = (int)(t % bk.nout);
    const int blk = blk0 + r;
    const int I = blk % bk.cx, J = (blk / bk.cx) % bk.cy, K = blk / (bk.cx * bk.cy);
    const int a = l % bk.nb, b = (l / bk.nb) % bk.nb, c = l / (bk.nb * bk.nb);
    const int64_t e = (bk.nb * I + a) + (int64_t)bk.nx * ((bk.nb * J + b) + (int64_t)bk.ny * (bk.nb * K + c));
    g[e] = (double)out[t];
  }
}

// rows idx[r] of D (clamped into [0, ns)) into rows r of A
__global__ void __launch_bounds__(TPB) gather_kernel(int B, int F, const int* __restrict__ idx, int ns,
                                                     const float* __restrict__ D, float* __restrict__ A) {
  const int64_t total = (int64_t)B * F;
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < total; t += (int64_t)gridDim.x * TPB) {
    const int r = (int)(t / F), f = (int)(t % F);
    int s = idx[r];
    s = s < 0 ? 0 : (s >= ns ? ns - 1 : s);
    A[t] = D[(int64_t)s * F + f];
  }
}

// Z (out x B, column-major) += bias, then ReLU unless this is the output layer
__global__ void __launch_bounds__(TPB) bias_act_kernel(int out, int B, const float* __restrict__ bias, int relu,
                                                       float* __restrict__ Z) {
  const int64_t total = (int64_t)out * B;
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < total; t += (int64_t)gridDim.x * TPB) {
    const float v = Z[t] + bias[t % out];
    Z[t] = relu ? fmaxf(v, 0.0f) : v;
  }
}

// dZ = 2 (P - Y) / (B out); the batch's loss mean((P - Y)^2) is summed in a
// fixed order by the single workgroup this kernel runs as (1024 threads,
// four independent loads in flight per thread).
__global__ void __launch_bounds__(1024) mse_kernel(int n, const float* __restrict__ P, const float* __restrict__ Y,
                                                   float* __restrict__ dZ, float* __restrict__ loss) {
  __shared__ double part[1024];
  double s = 0.0;
  const float sc = 2.0f / (float)n;
  int t = threadIdx.x;
  for (; t + 3 * 1024 < n; t += 4 * 1024) {
    float d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = P[t + k * 1024] - Y[t + k * 1024];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      dZ[t + k * 1024] = sc * d[k];
      s += (double)d[k] * (double)d[k];
    }
  }
  for (; t < n; t += 1024) {
    const float d = P[t] - Y[t];
    dZ[t] = sc * d;
    s += (double)d * (double)d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = (float)(part[0] / n);
}

// db[o] = sum over the batch of dZ[o, b]: a workgroup takes 16 outputs, its
// 16 slices of threads each sum every 16th sample (b = q, q + 16, ...), and
// the slices are added in q order (a fixed order throughout)
__global__ void __launch_bounds__(256) bias_grad_kernel(int out, int B, const float* __restrict__ dZ,
                                                        float* __restrict__ db) {
  __shared__ float part[16][16];
  const int ol = threadIdx.x % 16, q = threadIdx.x / 16;
  const int o = blockIdx.x * 16 + ol;
  float s = 0.0f;
  if (o < out) {
    int b = q;
    for (; b + 3 * 16 < B; b += 4 * 16) {
      float v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = dZ[(int64_t)(b + 16 * k) * out + o];
#pragma unroll
      for (int k = 0; k < 4; ++k) s += v[k];
    }
    for (; b < B; b += 16) s += dZ[(int64_t)b * out + o];
  }
  part[q][ol] = s;
  __syncthreads();
  if (q == 0 && o < out) {
    float t = 0.0f;
    for (int k = 0; k < 16; ++k) t += part[k][ol];
    db[o] = t;
  }
}

// dZ = dA where the layer's output was positive, else 0
__global__ void __launch_bounds__(TPB) relu_mask_kernel(int64_t n, const float* __restrict__ A,
                                                        float* __restrict__ dA) {
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TPB)
    if (!(A[t] > 0.0f)) dA[t] = 0.0f;
}

// Adam with bias correction: m, v moments; step size lr_t
__global__ void __launch_bounds__(TPB) adam_kernel(int64_t n, const float* __restrict__ g, float* __restrict__ p,
                                                   float* __restrict__ m, float* __restrict__ v, float b1, float b2,
                                                   float c1, float c2, float lr, float eps) {
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TPB) {
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
  }
}

__global__ void __launch_bounds__(TPB) to_float_kernel(int64_t n, const double* __restrict__ a,
                                                       float* __restrict__ b) {
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TPB) b[t] = (float)a[t];
}

__global__ void __launch_bounds__(TPB) to_double_kernel(int64_t n, const float* __restrict__ a,
                                                        double* __restrict__ b) {
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TPB) b[t] = (double)a[t];
}

__global__ void __launch_bounds__(TPB) fill_kernel(int64_t n, float* __restrict__ a) {
  for (int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TPB) a[t] = 0.0f;
}

struct Dims {
  int size[NL + 1];
  int64_t wofs[NL], bofs[NL], np;
};

Dims make_dims(int nb, int width) {
  Dims d;
  d.size[0] = nb * nb * nb + 24;
  for (int l = 1; l < NL; ++l) d.size[l] = width;
  d.size[NL] = nb * nb * nb;
  int64_t k = 0;
  for (int l = 0; l < NL; ++l) {
    d.wofs[l] = k;
    k += (int64_t)d.size[l] * d.size[l + 1];
    d.bofs[l] = k;
    k += d.size[l + 1];
  }
  d.np = k;
  return d;
}

constexpr size_t kAl = 256;
inline size_t al(size_t x) { return (x + kAl - 1) & ~(kAl - 1); }

}  // namespace

struct fe_onsg {
  Blocks bk;
  Dims dm;
  int width = 0, batch = 0, max_samples = 0, n_samples = 0;
  double* scales = nullptr;    // device: max |u_C| and max |g| of the current call
  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // parameters, gradient, Adam moments
  float *DX = nullptr, *DY = nullptr;                           // training samples
  float* A[NL + 1] = {};                                        // activations of a batch (A[0] = inputs)
  float *Yb = nullptr, *dZ = nullptr, *dA = nullptr;            // batch targets, back-propagated errors
};

namespace {

// One pass over the workspace: with base == nullptr it only measures.
size_t onsg_layout(const Blocks& bk, const Dims& dm, int max_samples, int batch, char* base, fe_onsg* o) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> float* {
    off = al(off);
    float* r = base ? reinterpret_cast<float*>(base + off) : nullptr;
    off += bytes;
    return r;
  };
  const size_t np = (size_t)dm.np;
  float* p = take(np * 4);
  float* g = take(np * 4);
  float* m = take(np * 4);
  float* v = take(np * 4);
  float* DX = take((size_t)max_samples * bk.nin * 4);
  float* DY = take((size_t)max_samples * bk.nout * 4);
  float* A[NL + 1];
  int wmax = 0;
  for (int l = 0; l <= NL; ++l) {
    A[l] = take((size_t)batch * dm.size[l] * 4);
    wmax = dm.size[l] > wmax ? dm.size[l] : wmax;
  }
  float* Yb = take((size_t)batch * bk.nout * 4);
  float* dZ = take((size_t)batch * wmax * 4);
  float* dA = take((size_t)batch * wmax * 4);
  float* sc = take(2 * sizeof(double));
  if (o) {
    o->p = p;
    o->g = g;
    o->m = m;
    o->v = v;
    o->DX = DX;
    o->DY = DY;
    for (int l = 0; l <= NL; ++l) o->A[l] = A[l];
    o->Yb = Yb;
    o->dZ = dZ;
    o->dA = dA;
    o->scales = reinterpret_cast<double*>(sc);
  }
  return al(off);
}

std::string onsg_validate(int nx, int ny, int nz, int nb, int width, int max_samples, int batch) {
  if (nx < 1 || ny < 1 || nz < 1) return "grid dimensions must be >= 1";
  if (nb < 1 || nx % nb || ny % nb || nz % nb) return "nb must be >= 1 and divide nx, ny and nz";
  if (nb > 16) return "nb must be <= 16";
  if (width < 1 || width > 8192) return "width must lie in [1, 8192]";
  if (batch < 1 || batch > 65536) return "batch must lie in [1, 65536]";
  if (max_samples < 1) return "max_samples must be >= 1";
  return "";
}

Blocks make_blocks(int nx, int ny, int nz, int nb) {
  Blocks b;
  b.nx = nx;
  b.ny = ny;
  b.nb = nb;
  b.cx = nx / nb;
  b.cy = ny / nb;
  b.nblk = (nx / nb) * (ny / nb) * (nz / nb);
  b.nin = nb * nb * nb + 24;
  b.nout = nb * nb * nb;
  return b;
}

#define ONSG_HIP(expr)                                                      \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      fe_set_error(std::string(#expr) + ": " + hipGetErrorString(e_));      \
      return FE_EDEVICE;                                                    \
    }                                                                       \
  } while (0)

#define ONSG_BLAS(expr)                                                     \
  do {                                                                      \
    rocblas_status s_ = (expr);                                             \
    if (s_ != rocblas_status_success) {                                     \
      fe_set_error(std::string(#expr) + ": " + rocblas_status_to_string(s_)); \
      return FE_EDEVICE;                                                    \
    }                                                                       \
  } while (0)

// Forward pass of rows A[0] (n <= batch): A[l+1] = act(W_l A[l] + b_l).
fe_status forward(fe_onsg* o, int n) {
  const float one = 1.0f, zero = 0.0f;
  for (int l = 0; l < NL; ++l) {
    const int in = o->dm.size[l], out = o->dm.size[l + 1];
    ONSG_BLAS(rocblas_sgemm(o->blas, rocblas_operation_transpose, rocblas_operation_none, out, n, in, &one,
                            o->p + o->dm.wofs[l], in, o->A[l], in, &zero, o->A[l + 1], out));
    hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for((int64_t)out * n)), dim3(TPB), 0, o->stream, out, n,
                       o->p + o->dm.bofs[l], l < NL - 1 ? 1 : 0, o->A[l + 1]);
    ONSG_HIP(hipGetLastError());
  }
  return FE_OK;
}

}  // namespace

extern "C" int64_t fe_onsg_num_params(int32_t nb, int32_t width) {
  if (nb < 1 || nb > 16 || width < 1 || width > 8192) return 0;
  return make_dims(nb, width).np;
}

extern "C" size_t fe_onsg_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t nb, int32_t width,
                                         int32_t max_samples, int32_t batch) {
  if (!onsg_validate(nx, ny, nz, nb, width, max_samples, batch).empty()) return 0;
  return onsg_layout(make_blocks(nx, ny, nz, nb), make_dims(nb, width), max_samples, batch, nullptr, nullptr);
}

extern "C" fe_status fe_onsg_create(int32_t nx, int32_t ny, int32_t nz, int32_t nb, int32_t width,
                                    int32_t max_samples, int32_t batch, const double* params, void* ws, size_t ws_bytes, void* stream_ptr,
                                    fe_onsg** out) {
  hipStream_t stream = static_cast<hipStream_t>(stream_ptr);
  if (!out || !params || !ws) {
    fe_set_error("out, params and ws must not be NULL");
    return FE_EINVAL;
  }
  *out = nullptr;
  const std::string why = onsg_validate(nx, ny, nz, nb, width, max_samples, batch);
  if (!why.empty()) {
    fe_set_error(why);
    return FE_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(ws) % kAl) {
    fe_set_error("ws must be 256-byte aligned");
    return FE_EINVAL;
  }
  const Blocks bk = make_blocks(nx, ny, nz, nb);
  const Dims dm = make_dims(nb, width);
  if (ws_bytes < onsg_layout(bk, dm, max_samples, batch, nullptr, nullptr)) {
    fe_set_error("workspace smaller than fe_onsg_workspace_size");
    return FE_ENOMEM;
  }
  fe_onsg* o = new fe_onsg();
  o->bk = bk;
  o->dm = dm;
  o->width = width;
  o->batch = batch;
  o->max_samples = max_samples;
  o->stream = stream;
  onsg_layout(bk, dm, max_samples, batch, static_cast<char*>(ws), o);
  if (rocblas_create_handle(&o->blas) != rocblas_status_success ||
      rocblas_set_stream(o->blas, stream) != rocblas_status_success) {
    if (o->blas) rocblas_destroy_handle(o->blas);
    delete o;
    fe_set_error("rocblas handle");
    return FE_EDEVICE;
  }
  hipLaunchKernelGGL(to_float_kernel, dim3(blocks_for(dm.np)), dim3(TPB), 0, stream, dm.np, params, o->p);
  if (hipGetLastError() != hipSuccess) {
    fe_onsg_destroy(o);
    fe_set_error("initial parameters");
    return FE_EDEVICE;
  }
  *out = o;
  return FE_OK;
}

extern "C" fe_status fe_onsg_add_samples(fe_onsg* o, const double* z, const double* uc, const double* g) {
  if (!o || !z || !uc || !g) {
    fe_set_error("handle, z, uc and g must not be NULL");
    return FE_EINVAL;
  }
  if (o->n_samples + o->bk.nblk > o->max_samples) {
    fe_set_error("training set full: max_samples reached");
    return FE_EINVAL;
  }
  const int64_t r0 = o->n_samples;
  const int64_t nuc = 3 * (int64_t)(o->bk.cx + 1) * (o->bk.cy + 1) * (o->bk.nblk / (o->bk.cx * o->bk.cy) + 1);
  const int64_t nel = (int64_t)o->bk.nblk * o->bk.nout;
  hipLaunchKernelGGL(absmax_kernel, dim3(1), dim3(1024), 0, o->stream, nuc, uc, o->scales);
  hipLaunchKernelGGL(absmax_kernel, dim3(1), dim3(1024), 0, o->stream, nel, g, o->scales + 1);
  hipLaunchKernelGGL(samples_kernel, dim3(blocks_for((int64_t)o->bk.nblk * o->bk.nin)), dim3(TPB), 0, o->stream,
                     o->bk, 0, o->bk.nblk, z, uc, g, o->scales, o->DX + r0 * o->bk.nin, o->DY + r0 * o->bk.nout);
  ONSG_HIP(hipGetLastError());
  o->n_samples += o->bk.nblk;
  return FE_OK;
}

extern "C" fe_status fe_onsg_num_samples(const fe_onsg* o, int64_t* n) {
  if (!o || !n) {
    fe_set_error("handle and n must not be NULL");
    return FE_EINVAL;
  }
  *n = o->n_samples;
  return FE_OK;
}

extern "C" fe_status fe_onsg_train(fe_onsg* o, int32_t steps, const int32_t* idx, double lr0, int32_t halve_every,
                                   float* losses) {
  if (!o || !idx || steps < 1 || halve_every < 1 || !(lr0 > 0.0)) {
    fe_set_error("need a handle, idx, steps >= 1, halve_every >= 1 and lr0 > 0");
    return FE_EINVAL;
  }
  if (o->n_samples < 1) {
    fe_set_error("no training samples");
    return FE_EINVAL;
  }
  const int B = o->batch, nin = o->bk.nin, nout = o->bk.nout;
  const int64_t np = o->dm.np;
  const float one = 1.0f, zero = 0.0f;
  const double b1 = 0.9, b2 = 0.999;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(np)), dim3(TPB), 0, o->stream, np, o->m);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(np)), dim3(TPB), 0, o->stream, np, o->v);
  ONSG_HIP(hipGetLastError());
  for (int t = 1; t <= steps; ++t) {
    const int* ix = idx + (int64_t)(t - 1) * B;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for((int64_t)B * nin)), dim3(TPB), 0, o->stream, B, nin, ix,
                       o->n_samples, o->DX, o->A[0]);
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for((int64_t)B * nout)), dim3(TPB), 0, o->stream, B, nout, ix,
                       o->n_samples, o->DY, o->Yb);
    ONSG_HIP(hipGetLastError());
    fe_status s = forward(o, B);
    if (s != FE_OK) return s;
    hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(1024), 0, o->stream, B * nout, o->A[NL], o->Yb, o->dZ,
                       losses ? losses + (t - 1) : nullptr);
    ONSG_HIP(hipGetLastError());
    for (int l = NL - 1; l >= 0; --l) {
      const int in = o->dm.size[l], out = o->dm.size[l + 1];
      // weight gradient (column-major in x out) = A_l dZ^T, bias gradient = row sums of dZ
      ONSG_BLAS(rocblas_sgemm(o->blas, rocblas_operation_none, rocblas_operation_transpose, in, out, B, &one,
                              o->A[l], in, o->dZ, out, &zero, o->g + o->dm.wofs[l], in));
      hipLaunchKernelGGL(bias_grad_kernel, dim3((out + 15) / 16), dim3(256), 0, o->stream, out, B, o->dZ,
                         o->g + o->dm.bofs[l]);
      ONSG_HIP(hipGetLastError());
      if (l > 0) {
        // error of the layer below: W^T dZ, masked where its ReLU was off
        ONSG_BLAS(rocblas_sgemm(o->blas, rocblas_operation_none, rocblas_operation_none, in, B, out, &one,
                                o->p + o->dm.wofs[l], in, o->dZ, out, &zero, o->dA, in));
        hipLaunchKernelGGL(relu_mask_kernel, dim3(blocks_for((int64_t)in * B)), dim3(TPB), 0, o->stream,
                           (int64_t)in * B, o->A[l], o->dA);
        ONSG_HIP(hipGetLastError());
        float* tmp = o->dZ;
        o->dZ = o->dA;
        o->dA = tmp;
      }
    }
    const double lr = lr0 * std::pow(0.5, (double)((t - 1) / halve_every));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(np)), dim3(TPB), 0, o->stream, np, o->g, o->p, o->m, o->v,
                       (float)b1, (float)b2, (float)(1.0 - std::pow(b1, t)), (float)(1.0 - std::pow(b2, t)),
                       (float)lr, 1e-8f);
    ONSG_HIP(hipGetLastError());
  }
  return FE_OK;
}

extern "C" fe_status fe_onsg_predict(fe_onsg* o, const double* z, const double* uc, double* g) {
  if (!o || !z || !uc || !g) {
    fe_set_error("handle, z, uc and g must not be NULL");
    return FE_EINVAL;
  }
  const int B = o->batch;
  const int64_t nuc = 3 * (int64_t)(o->bk.cx + 1) * (o->bk.cy + 1) * (o->bk.nblk / (o->bk.cx * o->bk.cy) + 1);
  hipLaunchKernelGGL(absmax_kernel, dim3(1), dim3(1024), 0, o->stream, nuc, uc, o->scales);
  for (int b0 = 0; b0 < o->bk.nblk; b0 += B) {
    const int n = o->bk.nblk - b0 < B ? o->bk.nblk - b0 : B;
    hipLaunchKernelGGL(samples_kernel, dim3(blocks_for((int64_t)n * o->bk.nin)), dim3(TPB), 0, o->stream, o->bk, b0,
                       n, z, uc, nullptr, o->scales, o->A[0], nullptr);
    ONSG_HIP(hipGetLastError());
    fe_status s = forward(o, n);
    if (s != FE_OK) return s;
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for((int64_t)n * o->bk.nout)), dim3(TPB), 0, o->stream, o->bk,
                       b0, n, o->A[NL], g);
    ONSG_HIP(hipGetLastError());
  }
  return FE_OK;
}

extern "C" fe_status fe_onsg_get_params(const fe_onsg* o, double* params) {
  if (!o || !params) {
    fe_set_error("handle and params must not be NULL");
    return FE_EINVAL;
  }
  hipLaunchKernelGGL(to_double_kernel, dim3(blocks_for(o->dm.np)), dim3(TPB), 0, o->stream, o->dm.np, o->p, params);
  ONSG_HIP(hipGetLastError());
  return FE_OK;
}

extern "C" void fe_onsg_destroy(fe_onsg* o) {
  if (!o) return;
  if (o->stream) (void)hipStreamSynchronize(o->stream);
  if (o->blas) rocblas_destroy_handle(o->blas);
  delete o;
}
