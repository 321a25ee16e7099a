// Pixel-domain steps of preconditioned conjugate gradient (Sec. II; the
// textbook iteration, Saad, "Iterative Methods for Sparse Linear Systems",
// Alg. 9.1) with the block-Jacobi M of eq. (7).
//
// Scalars (rho, alpha, beta, ||b||, the iteration count and a "done" flag)
// live in device memory, so a chunk of iterations is enqueued without host
// round trips; every kernel returns at once when "done" is set.  Dot products
// are deterministic: a fixed grid of kPcgBlocks blocks with a fixed pixel
// assignment writes per-block partials, and the last block to finish (an
// atomic ticket) sums them in a fixed order.
#include "mm_internal.h"

namespace mm {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum of two values; result valid in thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid] = a;
    sh[8 + wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a += sh[w];
      b += sh[8 + w];
    }
  }
}

// Write this block's two partials; returns true in every thread of the last
// block, whose thread 0 then holds the grid totals in (a, b).
__device__ bool grid_sum2(double& a, double& b, double* partials, uint32_t* counter, double* sh, bool* s_last) {
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = a;
    partials[kPcgBlocks + blockIdx.x] = b;
    __threadfence();
    const uint32_t ticket = atomicAdd(counter, 1u);
    *s_last = ticket == gridDim.x - 1;
  }
  __syncthreads();
  if (!*s_last) return false;
  __threadfence();
  double pa = 0.0, pb = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) {
    pa += partials[i];
    pb += partials[kPcgBlocks + i];
  }
  __syncthreads();
  block_sum2(pa, pb, sh);
  if (threadIdx.x == 0) {
    a = pa;
    b = pb;
    *counter = 0;
  }
  return true;
}

__device__ __forceinline__ void apply_m3(const double* __restrict__ m, double r0, double r1, double r2,
                                         double& z0, double& z1, double& z2) {
  z0 = m[0] * r0 + m[1] * r1 + m[2] * r2;
  z1 = m[1] * r0 + m[3] * r1 + m[4] * r2;
  z2 = m[2] * r0 + m[4] * r1 + m[5] * r2;
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_init(int32_t n_kept, const double* __restrict__ minv,
                                                          const double* __restrict__ b, double* __restrict__ x,
                                                          double* __restrict__ r, double* __restrict__ z,
                                                          double* __restrict__ p, double* __restrict__ q,
                                                          double* __restrict__ partials, PcgState* st,
                                                          double* __restrict__ hist, int32_t hist_len, double tol,
                                                          int32_t max_iter, int32_t fixed_iter) {
  __shared__ double sh[16];
  __shared__ bool s_last;
  double bb = 0.0, rz = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_kept; k += (int64_t)gridDim.x * blockDim.x) {
    const double b0 = b[3 * k], b1 = b[3 * k + 1], b2 = b[3 * k + 2];
    double z0, z1, z2;
    apply_m3(minv + 6 * k, b0, b1, b2, z0, z1, z2);
    x[3 * k] = 0.0; x[3 * k + 1] = 0.0; x[3 * k + 2] = 0.0;
    r[3 * k] = b0; r[3 * k + 1] = b1; r[3 * k + 2] = b2;
    z[3 * k] = z0; z[3 * k + 1] = z1; z[3 * k + 2] = z2;
    p[3 * k] = z0; p[3 * k + 1] = z1; p[3 * k + 2] = z2;
    q[3 * k] = 0.0; q[3 * k + 1] = 0.0; q[3 * k + 2] = 0.0;
    bb += b0 * b0 + b1 * b1 + b2 * b2;
    rz += b0 * z0 + b1 * z1 + b2 * z2;
  }
  if (!grid_sum2(bb, rz, partials, &st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    const double bnorm = sqrt(bb);
    const double rel = bnorm > 0.0 ? 1.0 : 0.0;
    st->rho = rz;
    st->alpha = 0.0;
    st->beta = 0.0;
    st->bnorm = bnorm;
    st->rel = rel;
    st->tol = tol;
    st->iter = 0;
    st->breakdown = 0;
    st->max_iter = max_iter;
    st->fixed_iter = fixed_iter;
    const bool met = rel <= tol;
    st->converged = met ? 1 : 0;
    st->done = (bnorm == 0.0 || (fixed_iter <= 0 && met) || (fixed_iter <= 0 && max_iter <= 0)) ? 1 : 0;
    if (fixed_iter > 0 && bnorm == 0.0) st->done = 1;
    if (hist_len > 0) hist[0] = rel;
  }
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_alpha(int32_t n_kept, const double* __restrict__ p,
                                                           const double* __restrict__ q,
                                                           double* __restrict__ partials, PcgState* st) {
  if (st->done) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  double pq = 0.0, unused = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)n_kept;
       i += (int64_t)gridDim.x * blockDim.x)
    pq += p[i] * q[i];
  if (!grid_sum2(pq, unused, partials, &st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    if (!(pq > 0.0) || isinf(pq)) {
      st->breakdown = 1;
      st->done = 1;
    } else {
      st->alpha = st->rho / pq;
    }
  }
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_update(int32_t n_kept, const double* __restrict__ minv,
                                                            double* __restrict__ x, double* __restrict__ r,
                                                            double* __restrict__ z, const double* __restrict__ p,
                                                            const double* __restrict__ q,
                                                            double* __restrict__ partials, PcgState* st,
                                                            double* __restrict__ hist, int32_t hist_len) {
  if (st->done) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  const double alpha = st->alpha;
  double rr = 0.0, rz = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_kept; k += (int64_t)gridDim.x * blockDim.x) {
    double rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[3 * k + c] += alpha * p[3 * k + c];
      rv[c] = r[3 * k + c] - alpha * q[3 * k + c];
      r[3 * k + c] = rv[c];
    }
    double z0, z1, z2;
    apply_m3(minv + 6 * k, rv[0], rv[1], rv[2], z0, z1, z2);
    z[3 * k] = z0; z[3 * k + 1] = z1; z[3 * k + 2] = z2;
    rr += rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    rz += rv[0] * z0 + rv[1] * z1 + rv[2] * z2;
  }
  if (!grid_sum2(rr, rz, partials, &st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    const int it = st->iter + 1;
    st->iter = it;
    const double rel = sqrt(rr) / st->bnorm;
    st->rel = rel;
    if (it < hist_len) hist[it] = rel;
    if (!isfinite(rel)) {
      st->breakdown = 1;
      st->done = 1;
    } else if (st->fixed_iter > 0) {
      if (it >= st->fixed_iter) {
        st->done = 1;
        st->converged = rel <= st->tol ? 1 : 0;
      }
    } else if (rel <= st->tol) {
      st->done = 1;
      st->converged = 1;
    } else if (it >= st->max_iter) {
      st->done = 1;
    }
    st->beta = rz / st->rho;
    st->rho = rz;
  }
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_direction(int32_t n_kept, const double* __restrict__ z,
                                                               double* __restrict__ p, double* __restrict__ q,
                                                               const PcgState* st) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)n_kept;
       i += (int64_t)gridDim.x * blockDim.x) {
    p[i] = z[i] + beta * p[i];
    q[i] = 0.0;
  }
}

// scratch0 = ||a - b||^2, scratch1 = ||a||^2
__global__ __launch_bounds__(kPcgThreads) void k_diff_norm(int64_t n, const double* __restrict__ a,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ partials, PcgState* st) {
  __shared__ double sh[16];
  __shared__ bool s_last;
  double dd = 0.0, aa = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = a[i] - b[i];
    dd += d * d;
    aa += a[i] * a[i];
  }
  if (!grid_sum2(dd, aa, partials, &st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    st->scratch0 = dd;
    st->scratch1 = aa;
  }
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] - b[i];
}

__global__ void k_add(int64_t n, double* __restrict__ y, const double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a[i];
}

}  // namespace

int launch_pcg_init(const mm_pointing_s* pt, PcgBufs& B, double tol, int32_t max_iter, int32_t fixed_iter,
                    hipStream_t s) {
  MM_HIP(hipMemsetAsync(&B.st->counter, 0, sizeof(uint32_t), s));
  hipLaunchKernelGGL(k_pcg_init, dim3(kPcgBlocks), dim3(kPcgThreads), 0, s, pt->n_kept, pt->minv, B.b, B.x, B.r, B.z,
                     B.p, B.q, B.partials, B.st, B.hist, B.hist_len, tol, max_iter, fixed_iter);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_pcg_iteration_tail(const mm_pointing_s* pt, PcgBufs& B, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_alpha, dim3(kPcgBlocks), dim3(kPcgThreads), 0, s, pt->n_kept, B.p, B.q, B.partials, B.st);
  hipLaunchKernelGGL(k_pcg_update, dim3(kPcgBlocks), dim3(kPcgThreads), 0, s, pt->n_kept, pt->minv, B.x, B.r, B.z,
                     B.p, B.q, B.partials, B.st, B.hist, B.hist_len);
  hipLaunchKernelGGL(k_pcg_direction, dim3(kPcgBlocks), dim3(kPcgThreads), 0, s, pt->n_kept, B.z, B.p, B.q, B.st);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_diff_norm(const mm_pointing_s* pt, const double* a, const double* b, PcgBufs& B, hipStream_t s) {
  hipLaunchKernelGGL(k_diff_norm, dim3(kPcgBlocks), dim3(kPcgThreads), 0, s, 3 * (int64_t)pt->n_kept, a, b,
                     B.partials, B.st);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_sub(const mm_pointing_s* pt, const double* a, const double* b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(kPcgBlocks), dim3(kPcgThreads), 0, s, 3 * (int64_t)pt->n_kept, a, b, y);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_add(const mm_pointing_s* pt, double* y, const double* a, hipStream_t s) {
  hipLaunchKernelGGL(k_add, dim3(kPcgBlocks), dim3(kPcgThreads), 0, s, 3 * (int64_t)pt->n_kept, y, a);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
