// Pixel-domain steps of preconditioned conjugate gradient (Sec. II; the
// textbook iteration, Saad, "Iterative Methods for Sparse Linear Systems",
// Alg. 9.1) with the block-Jacobi M of eq. (7), and the outer FP64
// refinement around an FP32-operator PCG.
//
// Every kernel runs one y-slice (blockIdx.y) per right-hand side; slice r
// uses the vectors at offset r * vstride, state st[r], partials
// [r * 2 * kPcgBlocks, ...) and history [r * hist_len, ...).  Scalars (rho,
// alpha, beta, ||b||, the iteration count, a "done" flag) live in device
// memory, so chunks of iterations are enqueued without host round trips and
// every kernel of a slice returns at once when that slice is done.  Dot
// products are deterministic: a fixed grid of kPcgBlocks blocks with a fixed
// pixel assignment writes per-block partials and the last block to finish
// (an atomic ticket) sums them in a fixed order.
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
// block of the slice, whose thread 0 then holds the slice totals in (a, b).
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

struct Slice {
  double *x, *r, *z, *p, *q;
  const double* b;
  double* partials;
  PcgState* st;
  double* hist;
};

__device__ __forceinline__ Slice slice(const PcgArgs& a) {
  const int64_t o = (int64_t)blockIdx.y * a.vstride;
  return Slice{a.x + o, a.r + o, a.z + o, a.p + o, a.q + o, a.b + o,
               a.partials + (int64_t)blockIdx.y * 2 * kPcgBlocks, a.st + blockIdx.y,
               a.hist + (int64_t)blockIdx.y * a.hist_len};
}

// x = 0, r = b, z = M r, p = z, q = 0, rho = r.z, ||b||.  Skipped for a
// slice whose gate (outer "done" flag) is set.
__global__ __launch_bounds__(kPcgThreads) void k_pcg_init(PcgArgs a, const double* __restrict__ minv, double tol,
                                                          int32_t max_iter, int32_t fixed_iter,
                                                          const OuterState* gate) {
  if (gate != nullptr && (gate[blockIdx.y].done || gate[blockIdx.y].skip)) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  Slice S = slice(a);
  double bb = 0.0, rz = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n_kept; k += (int64_t)gridDim.x * blockDim.x) {
    const double b0 = S.b[3 * k], b1 = S.b[3 * k + 1], b2 = S.b[3 * k + 2];
    double z0, z1, z2;
    apply_m3(minv + 6 * k, b0, b1, b2, z0, z1, z2);
    S.x[3 * k] = 0.0; S.x[3 * k + 1] = 0.0; S.x[3 * k + 2] = 0.0;
    S.r[3 * k] = b0; S.r[3 * k + 1] = b1; S.r[3 * k + 2] = b2;
    S.z[3 * k] = z0; S.z[3 * k + 1] = z1; S.z[3 * k + 2] = z2;
    S.p[3 * k] = z0; S.p[3 * k + 1] = z1; S.p[3 * k + 2] = z2;
    S.q[3 * k] = 0.0; S.q[3 * k + 1] = 0.0; S.q[3 * k + 2] = 0.0;
    bb += b0 * b0 + b1 * b1 + b2 * b2;
    rz += b0 * z0 + b1 * z1 + b2 * z2;
  }
  if (!grid_sum2(bb, rz, S.partials, &S.st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    PcgState* st = S.st;
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
    if (a.hist_len > 0) S.hist[0] = rel;
  }
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_alpha(PcgArgs a) {
  Slice S = slice(a);
  if (S.st->done) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  double pq = 0.0, unused = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)a.n_kept;
       i += (int64_t)gridDim.x * blockDim.x)
    pq += S.p[i] * S.q[i];
  if (!grid_sum2(pq, unused, S.partials, &S.st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    if (!(pq > 0.0) || isinf(pq)) {
      S.st->breakdown = 1;
      S.st->done = 1;
    } else {
      S.st->alpha = S.st->rho / pq;
    }
  }
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_update(PcgArgs a, const double* __restrict__ minv) {
  Slice S = slice(a);
  if (S.st->done) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  const double alpha = S.st->alpha;
  double rr = 0.0, rz = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n_kept; k += (int64_t)gridDim.x * blockDim.x) {
    double rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      S.x[3 * k + c] += alpha * S.p[3 * k + c];
      rv[c] = S.r[3 * k + c] - alpha * S.q[3 * k + c];
      S.r[3 * k + c] = rv[c];
    }
    double z0, z1, z2;
    apply_m3(minv + 6 * k, rv[0], rv[1], rv[2], z0, z1, z2);
    S.z[3 * k] = z0; S.z[3 * k + 1] = z1; S.z[3 * k + 2] = z2;
    rr += rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    rz += rv[0] * z0 + rv[1] * z1 + rv[2] * z2;
  }
  if (!grid_sum2(rr, rz, S.partials, &S.st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    PcgState* st = S.st;
    const int it = st->iter + 1;
    st->iter = it;
    const double rel = sqrt(rr) / st->bnorm;
    st->rel = rel;
    if (it < a.hist_len) S.hist[it] = rel;
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

__global__ __launch_bounds__(kPcgThreads) void k_pcg_direction(PcgArgs a) {
  Slice S = slice(a);
  if (S.st->done) return;
  const double beta = S.st->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)a.n_kept;
       i += (int64_t)gridDim.x * blockDim.x) {
    S.p[i] = S.z[i] + beta * S.p[i];
    S.q[i] = 0.0;
  }
}

// ---- outer FP64 refinement (per slice) ------------------------------------
// init: xt = 0, rt = b64, ||b64||; the inner state starts "done" so that
// nothing runs for a slice until its first inner solve is initialised.
__global__ __launch_bounds__(kPcgThreads) void k_outer_init(OuterArgs o, PcgArgs a) {
  __shared__ double sh[16];
  __shared__ bool s_last;
  const int64_t off = (int64_t)blockIdx.y * o.vstride;
  const int64_t n3 = 3 * (int64_t)a.n_kept;
  OuterState* os = o.os + blockIdx.y;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.st[blockIdx.y].done = 1;
    a.st[blockIdx.y].iter = 0;
    a.st[blockIdx.y].breakdown = 0;
  }
  double bb = 0.0, unused = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = o.b64[off + i];
    o.xt[off + i] = 0.0;
    o.rt[off + i] = v;
    bb += v * v;
  }
  if (!grid_sum2(bb, unused, o.partials + (int64_t)blockIdx.y * 2 * kPcgBlocks, &os->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    os->bnorm = sqrt(bb);
    os->rel = os->bnorm > 0.0 ? 1.0 : 0.0;
    os->iters = 0;
    os->inner_total = 0;
    os->converged = os->bnorm == 0.0 ? 1 : 0;
    os->done = os->bnorm == 0.0 ? 1 : 0;
    os->skip = 0;  // the first inner solve may start
    os->breakdown = 0;
  }
}

// A slice whose inner solve has ended and whose outer loop is still open
// takes an outer step: xt += x; q := 0 (A64 xt accumulates into q next).
__global__ __launch_bounds__(kPcgThreads) void k_outer_add(OuterArgs o, PcgArgs a) {
  const int64_t off = (int64_t)blockIdx.y * o.vstride;
  OuterState* os = o.os + blockIdx.y;
  const PcgState* st = a.st + blockIdx.y;
  const bool act = st->done && !os->done;
  if (!act) {
    if (blockIdx.x == 0 && threadIdx.x == 0) os->skip = 1;
    return;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)a.n_kept;
       i += (int64_t)gridDim.x * blockDim.x) {
    o.xt[off + i] += a.x[off + i];
    a.q[off + i] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    os->skip = 0;
    os->inner_total += st->iter;
    if (st->breakdown) os->breakdown = 1;
  }
}

// rt = b64 - q (q = A64 xt), ||rt|| / ||b64||, the outer stopping test.
__global__ __launch_bounds__(kPcgThreads) void k_outer_end(OuterArgs o, PcgArgs a, double tol, int32_t max_outer) {
  OuterState* os = o.os + blockIdx.y;
  if (os->skip) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  const int64_t off = (int64_t)blockIdx.y * o.vstride;
  double rr = 0.0, unused = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)a.n_kept;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = o.b64[off + i] - a.q[off + i];
    o.rt[off + i] = v;
    rr += v * v;
  }
  if (!grid_sum2(rr, unused, o.partials + (int64_t)blockIdx.y * 2 * kPcgBlocks, &os->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    const int it = os->iters + 1;
    os->iters = it;
    const double rel = sqrt(rr) / os->bnorm;
    os->rel = rel;
    if (it < o.hist_len) o.hist[(int64_t)blockIdx.y * o.hist_len + it] = rel;
    if (rel <= tol) {
      os->converged = 1;
      os->done = 1;
    } else if (it >= max_outer || os->breakdown || !isfinite(rel)) {
      os->done = 1;
    }
  }
}

// scratch0 = ||a - b||^2, scratch1 = ||a||^2 per slice
__global__ __launch_bounds__(kPcgThreads) void k_diff_norm(PcgArgs A, const double* __restrict__ a,
                                                           const double* __restrict__ b) {
  __shared__ double sh[16];
  __shared__ bool s_last;
  Slice S = slice(A);
  const int64_t off = (int64_t)blockIdx.y * A.vstride;
  double dd = 0.0, aa = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)A.n_kept;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = a[off + i] - b[off + i];
    dd += d * d;
    aa += a[off + i] * a[off + i];
  }
  if (!grid_sum2(dd, aa, S.partials, &S.st->counter, sh, &s_last)) return;
  if (threadIdx.x == 0) {
    S.st->scratch0 = dd;
    S.st->scratch1 = aa;
  }
}

}  // namespace

int launch_pcg_init(const mm_pointing_s* pt, const PcgArgs& a, int nrhs, double tol, int32_t max_iter,
                    int32_t fixed_iter, const OuterState* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_init, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, a, pt->minv, tol, max_iter,
                     fixed_iter, gate);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_pcg_iteration_tail(const mm_pointing_s* pt, const PcgArgs& a, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_alpha, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, a);
  hipLaunchKernelGGL(k_pcg_update, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, a, pt->minv);
  hipLaunchKernelGGL(k_pcg_direction, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, a);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_diff_norm(const PcgArgs& a, int nrhs, const double* x, const double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_diff_norm, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, a, x, y);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_init(const OuterArgs& o, const PcgArgs& a, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_init, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, o, a);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_add(const OuterArgs& o, const PcgArgs& a, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_add, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, o, a);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_end(const OuterArgs& o, const PcgArgs& a, int nrhs, double tol, int32_t max_outer,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_outer_end, dim3(kPcgBlocks, nrhs), dim3(kPcgThreads), 0, s, o, a, tol, max_outer);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
