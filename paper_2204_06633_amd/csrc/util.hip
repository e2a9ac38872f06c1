// Small helper kernels: zero fill (graph-safe replacement of memset nodes)
// and the fixed-order reduction of per-workgroup sky-gradient partials.
#include "internal.hpp"

namespace lr {

__global__ void fill_zero_kernel(double* p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0.0;
}

// Sum the per-workgroup sky partials in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void sky_finalize_kernel(const double* part, int64_t nblocks,
                                                           double* g_sky) {
  __shared__ double s[2][256];
  const int tid = threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t b = tid; b < nblocks; b += 256) { a0 += part[2 * b]; a1 += part[2 * b + 1]; }
  s[0][tid] = a0;
  s[1][tid] = a1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) { s[0][tid] += s[0][tid + w]; s[1][tid] += s[1][tid + w]; }
    __syncthreads();
  }
  if (tid == 0) { g_sky[0] = s[0][0]; g_sky[1] = s[1][0]; }
}

// White-noise Gaussian log-likelihood pieces (Sec. II.A, eq. like, summed over
// channels as in Sec. IV.C): per-workgroup partial sums of (d - h)^2 and,
// optionally, the gradient (d - h)/sigma^2 with respect to h.  A fixed grid
// and a fixed per-lane order keep the sum deterministic.
constexpr int kLikeBlocks = 1024;

__global__ __launch_bounds__(256) void loglike_kernel(const double* h, const double* d, int64_t n,
                                                      double inv_var, double* g, double* part) {
  __shared__ double s[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t k = (int64_t)blockIdx.x * 256 + tid; k < n; k += stride) {
    const double r = d[k] - h[k];
    acc = fma(r, r, acc);
    if (g) g[k] = r * inv_var;
  }
  s[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) s[tid] += s[tid + w];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void loglike_finalize_kernel(const double* part, int nblocks,
                                                               double inv_var, double* out) {
  __shared__ double s[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int b = tid; b < nblocks; b += 256) acc += part[b];
  s[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) s[tid] += s[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[0] = -0.5 * inv_var * s[0];
}

size_t loglike_workspace_bytes() { return kLikeBlocks * sizeof(double); }

hipError_t run_loglike(const double* h, const double* d, int64_t n, double inv_var, double* g,
                       double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(loglike_kernel, dim3(kLikeBlocks), dim3(256), 0, s, h, d, n, inv_var, g, part);
  hipLaunchKernelGGL(loglike_finalize_kernel, dim3(1), dim3(256), 0, s, part, kLikeBlocks, inv_var,
                     out);
  return hipGetLastError();
}

// Batched likelihood: items are element ranges [begin, end) of one
// template's output block; the finalisation sums each template's item
// partials in order.
__global__ __launch_bounds__(256) void batch_loglike_kernel(const double* h, const double* d,
                                                            const int64_t* items, double inv_var,
                                                            double* g, double* part) {
  __shared__ double s[256];
  const int tid = threadIdx.x;
  const int64_t b0 = items[2 * blockIdx.x], b1 = items[2 * blockIdx.x + 1];
  double acc = 0.0;
  for (int64_t k = b0 + tid; k < b1; k += 256) {
    const double r = d[k] - h[k];
    acc = fma(r, r, acc);
    if (g) g[k] = r * inv_var;
  }
  s[tid] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) s[tid] += s[tid + w];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = s[0];
}

// One workgroup per template: out[index] = -1/2 inv_var * sum of its partials
// (pairs: first item, item count, output index).
__global__ __launch_bounds__(256) void batch_finalize_kernel(const double* part, int width,
                                                             const int64_t* span,
                                                             double scale, double* out) {
  __shared__ double s[2][256];
  const int tid = threadIdx.x;
  const int64_t first = span[3 * blockIdx.x], count = span[3 * blockIdx.x + 1];
  const int64_t index = span[3 * blockIdx.x + 2];
  double a0 = 0.0, a1 = 0.0;
  for (int64_t k = tid; k < count; k += 256) {
    a0 += part[width * (first + k)];
    if (width > 1) a1 += part[width * (first + k) + 1];
  }
  s[0][tid] = a0;
  s[1][tid] = a1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) { s[0][tid] += s[0][tid + w]; s[1][tid] += s[1][tid + w]; }
    __syncthreads();
  }
  if (tid == 0) {
    out[width * index] = scale * s[0][0];
    if (width > 1) out[width * index + 1] = scale * s[1][0];
  }
}

hipError_t run_batch_loglike(const double* h, const double* d, const int64_t* items,
                             int64_t n_items, double inv_var, double* g, double* part,
                             const int64_t* span, int64_t n_templates, double* out,
                             hipStream_t s) {
  if (n_items > 0)
    hipLaunchKernelGGL(batch_loglike_kernel, dim3((unsigned)n_items), dim3(256), 0, s, h, d,
                       items, inv_var, g, part);
  hipLaunchKernelGGL(batch_finalize_kernel, dim3((unsigned)n_templates), dim3(256), 0, s, part,
                     1, span, -0.5 * inv_var, out);
  return hipGetLastError();
}

hipError_t run_batch_sky_finalize(const double* part, const int64_t* span, int64_t n_templates,
                                  double* g_sky, hipStream_t s) {
  hipLaunchKernelGGL(batch_finalize_kernel, dim3((unsigned)n_templates), dim3(256), 0, s, part, 2,
                     span, 1.0, g_sky);
  return hipGetLastError();
}

__global__ void forward_prep_kernel(int* counter, const double* sky, int stride, int64_t n,
                                    double* trig) {
  const int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (k == 0) *counter = 0;
  if (k < n) {
    double sn, cs;
    sincos(sky[stride * k], &sn, &cs);
    trig[4 * k] = sn;
    trig[4 * k + 1] = cs;
    sincos(sky[stride * k + 1], &sn, &cs);
    trig[4 * k + 2] = sn;
    trig[4 * k + 3] = cs;
  }
}

hipError_t run_forward_prep(int* counter, const double* sky, int stride, int64_t n,
                            double* trig, hipStream_t s) {
  const int64_t blocks = n > 0 ? (n + 63) / 64 : 1;
  hipLaunchKernelGGL(forward_prep_kernel, dim3((unsigned)blocks), dim3(64), 0, s, counter, sky,
                     stride, n, trig);
  return hipGetLastError();
}

hipError_t run_fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t run_sky_finalize(const double* part, int64_t nblocks, double* g_sky, hipStream_t s) {
  hipLaunchKernelGGL(sky_finalize_kernel, dim3(1), dim3(256), 0, s, part, nblocks, g_sky);
  return hipGetLastError();
}

}  // namespace lr
