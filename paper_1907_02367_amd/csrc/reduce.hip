// Deterministic FP64 reductions over the stored point values:
//   kind 0: error of Sec. 6 on the flat front t = T against exact values,
//           sum w (c^-2 (v - v_ex)^2 + |sigma - sigma_ex|^2) and the same norm of
//           the exact values;
//   kind 1: energy on the current front (Sec. 6.5 in flux form),
//           1/2 sum w (c^-2 v^2 + |sigma|^2 - 2 v sigma.grad phi);
//   kind 2: L2 error of U on the flat front (Sec. 6.6) against exact values,
//           sum w (U - U_ex)^2 and sum w U_ex^2.
// Two passes: fixed grid of blocks -> per-block partial sums (tree order),
// then one block sums the partials in a fixed order.  No floating-point atomics.
#include <hip/hip_runtime.h>

#include "tdg_internal.h"

namespace tdg {

namespace {

constexpr int kRB = 256;

__device__ inline void block_sum2(double& a, double& b, double* sh) {
  sh[threadIdx.x] = a;
  sh[kRB + threadIdx.x] = b;
  __syncthreads();
  for (int s = kRB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sh[threadIdx.x] += sh[threadIdx.x + s];
      sh[kRB + threadIdx.x] += sh[kRB + threadIdx.x + s];
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[kRB];
}

template <int NS>
__global__ __launch_bounds__(kRB) void norms_kernel(KParams P, int kind, const double* ex, double* partial) {
  __shared__ double sh[2 * kRB];
  const int Q = P.Q;
  const long long nq = (long long)P.ne * Q;
  double s0 = 0.0, s1 = 0.0;
  for (long long i = (long long)blockIdx.x * kRB + threadIdx.x; i < nq; i += (long long)gridDim.x * kRB) {
    const int e = (int)(i / Q), q = (int)(i % Q);
    const double w = P.w_ref[q] * P.absdet[e];
    const double ic2 = 1.0 / (P.c[e] * P.c[e]);
    const double* st = P.state + (size_t)e * (NS + 2) * Q;
    const double v = st[q];
    if (kind == 0) {
      const double dv = v - ex[i];
      double a = ic2 * dv * dv, b = ic2 * ex[i] * ex[i];
      for (int d = 0; d < NS; ++d) {
        const double se = ex[nq + i * NS + d];
        const double ds = st[(1 + d) * Q + q] - se;
        a += ds * ds;
        b += se * se;
      }
      s0 += w * a;
      s1 += w * b;
    } else if (kind == 2) {
      const double du = st[(NS + 1) * Q + q] - ex[i];
      s0 += w * du * du;
      s1 += w * ex[i] * ex[i];
    } else {
      const int* vs = P.elems + (size_t)e * (NS + 1);
      const double* gl = P.grad_lam + (size_t)e * (NS + 1) * NS;
      double dens = ic2 * v * v;
      for (int d = 0; d < NS; ++d) {
        double g = 0.0;
        for (int k = 0; k <= NS; ++k) g += P.tau[vs[k]] * gl[k * NS + d];
        const double s = st[(1 + d) * Q + q];
        dens += s * s - 2.0 * v * s * g;
      }
      s0 += 0.5 * w * dens;
    }
  }
  block_sum2(s0, s1, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0;
    partial[2 * blockIdx.x + 1] = s1;
  }
}

__global__ __launch_bounds__(kRB) void sum_partials(const double* partial, int nblocks, double* out) {
  __shared__ double sh[2 * kRB];
  double s0 = 0.0, s1 = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += kRB) {
    s0 += partial[2 * i];
    s1 += partial[2 * i + 1];
  }
  block_sum2(s0, s1, sh);
  if (threadIdx.x == 0) {
    out[0] = s0;
    out[1] = s1;
  }
}

__global__ void fill_kernel(double* p, double v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_i8_kernel(signed char* p, signed char v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

int launch_norms(const KParams& P, int kind, const double* ex, double* partial, int nblocks, double* out,
                 void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  switch (P.n) {
    case 1:
      hipLaunchKernelGGL(norms_kernel<1>, dim3(nblocks), dim3(kRB), 0, stream, P, kind, ex, partial);
      break;
    case 2:
      hipLaunchKernelGGL(norms_kernel<2>, dim3(nblocks), dim3(kRB), 0, stream, P, kind, ex, partial);
      break;
    default:
      hipLaunchKernelGGL(norms_kernel<3>, dim3(nblocks), dim3(kRB), 0, stream, P, kind, ex, partial);
      break;
  }
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(kRB), 0, stream, partial, nblocks, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill(double* p, double v, long long n, void* stream_) {
  if (n <= 0) return 0;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream_, p, v, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fill_i8(signed char* p, signed char v, long long n, void* stream_) {
  if (n <= 0) return 0;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_i8_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream_, p, v, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tdg
