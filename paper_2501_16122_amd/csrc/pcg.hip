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
// products are deterministic: a block count fixed by the problem size
// (pcg_blocks) with a fixed pixel assignment writes per-block partials and
// the last block to finish (an atomic ticket) sums them in a fixed order.
// A batched launch spans the largest member's block count; blocks past a
// member's own count return at once, so a member's sums, and its iterates,
// are the same alone and in any batch.
#include <algorithm>

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
__device__ bool grid_sum2(double& a, double& b, double* partials, uint32_t* counter, double* sh, bool* s_last,
                          int nblk) {
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = a;
    partials[kPcgBlocks + blockIdx.x] = b;
    __threadfence();
    const uint32_t ticket = atomicAdd(counter, 1u);
    *s_last = ticket == (uint32_t)nblk - 1;
  }
  __syncthreads();
  if (!*s_last) return false;
  __threadfence();
  double pa = 0.0, pb = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
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

// z = B^-1 r for one pixel: the symmetric NC x NC inverse block of eq. (7)
// stored as its upper triangle, row-major.
template <int NC>
__device__ __forceinline__ void apply_m(const double* __restrict__ m, const double* r, double* z) {
  if constexpr (NC == 3) {
    z[0] = m[0] * r[0] + m[1] * r[1] + m[2] * r[2];
    z[1] = m[1] * r[0] + m[3] * r[1] + m[4] * r[2];
    z[2] = m[2] * r[0] + m[4] * r[1] + m[5] * r[2];
  } else if constexpr (NC == 2) {
    z[0] = m[0] * r[0] + m[1] * r[1];
    z[1] = m[1] * r[0] + m[2] * r[1];
  } else {
    z[0] = m[0] * r[0];
  }
}

// One right-hand side: its vectors, state, partials and history.
struct Slice {
  double *x, *r, *z, *p, *q;
  const double* b;
  double* partials;
  PcgState* st;
  double* hist;
  int32_t n_kept;
  int32_t hist_len;
  int32_t ncomp;  // values per kept pixel
  int64_t n;      // ncomp * n_kept values per vector
  int32_t nblk;   // blocks that work on this right-hand side (pcg_blocks)
};

__device__ __forceinline__ Slice slice(const PcgArgs& a, int y) {
  const int64_t o = (int64_t)y * a.vstride;
  return Slice{a.x + o, a.r + o, a.z + o, a.p + o, a.q + o, a.b + o,
               a.partials + (int64_t)y * 2 * kPcgBlocks, a.st + y, a.hist + (int64_t)y * a.hist_len,
               a.n_kept, a.hist_len, a.ncomp, (int64_t)a.ncomp * a.n_kept, pcg_blocks(a.n_kept)};
}

// The outer refinement vectors and state of one right-hand side.
struct OSlice {
  double *xt, *rt;
  const double* b64;
  double* partials;
  OuterState* os;
  double* hist;
  int32_t hist_len;
};

__device__ __forceinline__ OSlice oslice(const OuterArgs& o, int y) {
  const int64_t off = (int64_t)y * o.vstride;
  return OSlice{o.xt + off, o.rt + off, o.b64 + off, o.partials + (int64_t)y * 2 * kPcgBlocks, o.os + y,
                o.hist + (int64_t)y * o.hist_len, o.hist_len};
}

// ---- bodies (one right-hand side each) ------------------------------------

// x = 0, r = b, z = M r, p = z, q = 0, rho = r.z, ||b||.  Skipped while the
// gate (outer state) is done or has no step pending.  From a start vector
// (from_x0): x already holds x0 and q holds A x0, so r = b - A x0 (x is
// reset to 0 when b = 0, whose solution is 0).
template <int NC>
__device__ __forceinline__ void pcg_init_sums(const Slice& S, const double* __restrict__ minv, bool from_x0,
                                              bool zero_b, double& bb, double& rz) {
  constexpr int NB = NC * (NC + 1) / 2;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < S.n_kept; k += (int64_t)S.nblk * blockDim.x) {
    double bv[NC], rv[NC], zv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bv[c] = S.b[NC * k + c];
      rv[c] = from_x0 ? bv[c] - S.q[NC * k + c] : bv[c];
    }
    apply_m<NC>(minv + NB * k, rv, zv);
    double sb = 0.0, sz = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t i = NC * k + c;
      if (!from_x0 || zero_b) S.x[i] = 0.0;
      S.r[i] = rv[c];
      S.z[i] = zv[c];
      S.p[i] = zv[c];
      S.q[i] = 0.0;
      sb += bv[c] * bv[c];
      sz += rv[c] * zv[c];
    }
    bb += sb;
    rz += sz;
  }
}

// from_x0: st->scratch0 = ||b - A x0||^2 and st->scratch1 = ||b||^2 were
// computed beforehand (launch_diff_norm).
__device__ __forceinline__ void pcg_init_body(const Slice& S, const double* __restrict__ minv, double tol,
                                              int32_t max_iter, int32_t fixed_iter, const OuterState* gate,
                                              bool from_x0 = false) {
  if ((int)blockIdx.x >= S.nblk) return;
  if (gate != nullptr && (gate->done || gate->skip)) return;
  // an inner solve of the refinement goes no deeper than the outer
  // tolerance needs: relative to its right-hand side r_k it must reach
  // tol ||b|| / ||r_k||, with a factor 2 to spare, and never less deep than
  // the inner tolerance
  if (gate != nullptr && gate->target > 0.0 && gate->rel > 0.0) tol = fmax(tol, 0.5 * gate->target / gate->rel);
  __shared__ double sh[16];
  __shared__ bool s_last;
  double bb = 0.0, rz = 0.0;
  const double r0 = from_x0 ? S.st->scratch0 : 0.0, b0 = from_x0 ? S.st->scratch1 : 0.0;
  const bool zero_b = from_x0 && !(b0 > 0.0);
  if (S.ncomp == 3) pcg_init_sums<3>(S, minv, from_x0, zero_b, bb, rz);
  else if (S.ncomp == 2) pcg_init_sums<2>(S, minv, from_x0, zero_b, bb, rz);
  else pcg_init_sums<1>(S, minv, from_x0, zero_b, bb, rz);
  if (!grid_sum2(bb, rz, S.partials, &S.st->counter, sh, &s_last, S.nblk)) return;
  if (threadIdx.x == 0) {
    PcgState* st = S.st;
    const double bnorm = sqrt(bb);
    const double rel = bnorm > 0.0 ? (from_x0 ? sqrt(r0) / bnorm : 1.0) : 0.0;
    st->rho = rz;
    st->alpha = 0.0;
    st->beta = 0.0;
    st->bnorm = bnorm;
    st->rel = rel;
    st->tol = tol;
    st->iter = 0;
    st->max_iter = max_iter;
    st->fixed_iter = fixed_iter;
    // a non-finite right-hand side, start residual or r.z is a breakdown
    const bool bad = !isfinite(bb) || !isfinite(rz) || !isfinite(rel);
    st->breakdown = bad ? 1 : 0;
    const bool met = !bad && rel <= tol;
    st->converged = met ? 1 : 0;
    st->done = (bad || bnorm == 0.0 || (fixed_iter <= 0 && met) || (fixed_iter <= 0 && max_iter <= 0)) ? 1 : 0;
    if (S.hist_len > 0) S.hist[0] = rel;
  }
}

// alpha = rho / p.q (breakdown if p.q <= 0 or not finite)
__device__ __forceinline__ void pcg_alpha_body(const Slice& S) {
  if ((int)blockIdx.x >= S.nblk || S.st->done) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  double pq = 0.0, unused = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)S.nblk * blockDim.x)
    pq += S.p[i] * S.q[i];
  if (!grid_sum2(pq, unused, S.partials, &S.st->counter, sh, &s_last, S.nblk)) return;
  if (threadIdx.x == 0) {
    if (!(pq > 0.0) || isinf(pq)) {
      S.st->breakdown = 1;
      S.st->done = 1;
    } else {
      S.st->alpha = S.st->rho / pq;
    }
  }
}

// x += alpha p, r -= alpha q, z = M r, ||r||, r.z, the stopping test, beta
template <int NC>
__device__ __forceinline__ void pcg_update_sums(const Slice& S, const double* __restrict__ minv, double alpha,
                                                double& rr, double& rz) {
  constexpr int NB = NC * (NC + 1) / 2;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < S.n_kept; k += (int64_t)S.nblk * blockDim.x) {
    double rv[NC], zv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t i = NC * k + c;
      S.x[i] += alpha * S.p[i];
      rv[c] = S.r[i] - alpha * S.q[i];
      S.r[i] = rv[c];
    }
    apply_m<NC>(minv + NB * k, rv, zv);
    double sr = 0.0, sz = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      S.z[NC * k + c] = zv[c];
      sr += rv[c] * rv[c];
      sz += rv[c] * zv[c];
    }
    rr += sr;
    rz += sz;
  }
}

__device__ __forceinline__ void pcg_update_body(const Slice& S, const double* __restrict__ minv) {
  if ((int)blockIdx.x >= S.nblk || S.st->done) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  const double alpha = S.st->alpha;
  double rr = 0.0, rz = 0.0;
  if (S.ncomp == 3) pcg_update_sums<3>(S, minv, alpha, rr, rz);
  else if (S.ncomp == 2) pcg_update_sums<2>(S, minv, alpha, rr, rz);
  else pcg_update_sums<1>(S, minv, alpha, rr, rz);
  if (!grid_sum2(rr, rz, S.partials, &S.st->counter, sh, &s_last, S.nblk)) return;
  if (threadIdx.x == 0) {
    PcgState* st = S.st;
    const int it = st->iter + 1;
    st->iter = it;
    const double rel = sqrt(rr) / st->bnorm;
    st->rel = rel;
    if (it < S.hist_len) S.hist[it] = rel;
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

// p = z + beta p, q = 0 (the next operator launch accumulates into q)
__device__ __forceinline__ void pcg_direction_body(const Slice& S) {
  if ((int)blockIdx.x >= S.nblk || S.st->done) return;
  const double beta = S.st->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)S.nblk * blockDim.x) {
    S.p[i] = S.z[i] + beta * S.p[i];
    S.q[i] = 0.0;
  }
}

// ---- outer FP64 refinement ------------------------------------------------
// init: xt = 0, rt = b64, ||b64||; the inner state starts "done" so that
// nothing runs until the first inner solve is initialised.  From a start
// vector (from_x0): xt already holds x0, q holds A64 x0 and the inner
// scratch1 ||b64||^2, so rt = b64 - A64 x0; ||rt||^2 (sum 2) gives the
// starting residual.
__device__ __forceinline__ void outer_init_body(const OSlice& O, const Slice& S, bool from_x0 = false) {
  if ((int)blockIdx.x >= S.nblk) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  const int64_t n3 = S.n;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.st->done = 1;
    S.st->iter = 0;
    S.st->breakdown = 0;
  }
  // with b64 = 0 (||b64||^2 in the inner scratch1, see launch_diff_norm) the solution is 0
  const bool zero_b = from_x0 && !(S.st->scratch1 > 0.0);
  double bb = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)S.nblk * blockDim.x) {
    const double v = O.b64[i];
    const double r = from_x0 && !zero_b ? v - S.q[i] : v;
    if (!from_x0 || zero_b) O.xt[i] = 0.0;
    O.rt[i] = r;
    bb += v * v;
    rr += r * r;
  }
  if (!grid_sum2(bb, rr, O.partials, &O.os->counter, sh, &s_last, S.nblk)) return;
  if (threadIdx.x == 0) {
    OuterState* os = O.os;
    os->bnorm = sqrt(bb);
    os->rel = os->bnorm > 0.0 ? (from_x0 ? sqrt(rr) / os->bnorm : 1.0) : 0.0;
    os->iters = 0;
    os->inner_total = 0;
    // a non-finite right-hand side or start residual is a breakdown
    const bool bad = !isfinite(bb) || !isfinite(rr);
    os->converged = (!bad && os->bnorm == 0.0) ? 1 : 0;
    os->done = (bad || os->bnorm == 0.0) ? 1 : 0;
    os->skip = 0;  // the first inner solve may start
    os->breakdown = bad ? 1 : 0;
    os->target = 0.0;  // set when an outer step ends
  }
}

// A right-hand side whose inner solve has ended and whose outer loop is
// still open takes an outer step: xt += x; q := 0 (A64 xt accumulates into
// q next).  Any other right-hand side is marked skip.
__device__ __forceinline__ void outer_add_body(const OSlice& O, const Slice& S) {
  if ((int)blockIdx.x >= S.nblk) return;
  OuterState* os = O.os;
  const PcgState* st = S.st;
  const bool act = st->done && !os->done;
  if (!act) {
    if (blockIdx.x == 0 && threadIdx.x == 0) os->skip = 1;
    return;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)S.nblk * blockDim.x) {
    O.xt[i] += S.x[i];
    S.q[i] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    os->skip = 0;
    os->inner_total += st->iter;
    if (st->breakdown) os->breakdown = 1;
  }
}

// rt = b64 - q (q = A64 xt), ||rt|| / ||b64||, the outer stopping test.
__device__ __forceinline__ void outer_end_body(const OSlice& O, const Slice& S, double tol, int32_t max_outer) {
  if ((int)blockIdx.x >= S.nblk) return;
  OuterState* os = O.os;
  if (os->skip) return;
  __shared__ double sh[16];
  __shared__ bool s_last;
  double rr = 0.0, unused = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)S.nblk * blockDim.x) {
    const double v = O.b64[i] - S.q[i];
    O.rt[i] = v;
    rr += v * v;
  }
  if (!grid_sum2(rr, unused, O.partials, &os->counter, sh, &s_last, S.nblk)) return;
  if (threadIdx.x == 0) {
    const int it = os->iters + 1;
    os->iters = it;
    const double rel = sqrt(rr) / os->bnorm;
    os->rel = rel;
    os->target = tol;
    if (it < O.hist_len) O.hist[it] = rel;
    if (rel <= tol) {
      os->converged = 1;
      os->done = 1;
    } else if (it >= max_outer || os->breakdown || !isfinite(rel)) {
      os->done = 1;
    }
  }
}

// ---- kernels: one slice per blockIdx.y -------------------------------------
// Single solver: slice blockIdx.y of one PcgArgs (a right-hand side).
// Batch: slot blockIdx.y of a PcgBatch (slice 0 of that slot's views).

__global__ __launch_bounds__(kPcgThreads) void k_pcg_init(PcgArgs a, const double* __restrict__ minv, double tol,
                                                          int32_t max_iter, int32_t fixed_iter,
                                                          const OuterState* gate, int32_t from_x0) {
  pcg_init_body(slice(a, blockIdx.y), minv, tol, max_iter, fixed_iter, gate ? gate + blockIdx.y : nullptr,
                from_x0 != 0);
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_alpha(PcgArgs a) { pcg_alpha_body(slice(a, blockIdx.y)); }

__global__ __launch_bounds__(kPcgThreads) void k_pcg_update(PcgArgs a, const double* __restrict__ minv) {
  pcg_update_body(slice(a, blockIdx.y), minv);
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_direction(PcgArgs a) {
  pcg_direction_body(slice(a, blockIdx.y));
}

__global__ __launch_bounds__(kPcgThreads) void k_outer_init(OuterArgs o, PcgArgs a, int32_t from_x0) {
  outer_init_body(oslice(o, blockIdx.y), slice(a, blockIdx.y), from_x0 != 0);
}

__global__ __launch_bounds__(kPcgThreads) void k_outer_add(OuterArgs o, PcgArgs a) {
  outer_add_body(oslice(o, blockIdx.y), slice(a, blockIdx.y));
}

__global__ __launch_bounds__(kPcgThreads) void k_outer_end(OuterArgs o, PcgArgs a, double tol, int32_t max_outer) {
  outer_end_body(oslice(o, blockIdx.y), slice(a, blockIdx.y), tol, max_outer);
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_alpha_b(PcgBatch b) {
  pcg_alpha_body(slice(b.s[blockIdx.y].A, 0));
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_update_b(PcgBatch b) {
  pcg_update_body(slice(b.s[blockIdx.y].A, 0), b.s[blockIdx.y].minv);
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_direction_b(PcgBatch b) {
  pcg_direction_body(slice(b.s[blockIdx.y].A, 0));
}

__global__ __launch_bounds__(kPcgThreads) void k_outer_add_b(PcgBatch b) {
  const PcgSlot& p = b.s[blockIdx.y];
  outer_add_body(oslice(p.O, 0), slice(p.A, 0));
}

__global__ __launch_bounds__(kPcgThreads) void k_outer_end_b(PcgBatch b) {
  const PcgSlot& p = b.s[blockIdx.y];
  outer_end_body(oslice(p.O, 0), slice(p.A, 0), p.tol, p.O.max_outer);
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg_reinit_b(PcgBatch b) {
  const PcgSlot& p = b.s[blockIdx.y];
  pcg_init_body(slice(p.A, 0), p.minv, p.inner_tol, p.A.max_iter, 0, p.O.os);
}

// scratch0 = ||a - b||^2, scratch1 = ||a||^2 per slice
__global__ __launch_bounds__(kPcgThreads) void k_diff_norm(PcgArgs A, const double* __restrict__ a,
                                                           const double* __restrict__ b) {
  __shared__ double sh[16];
  __shared__ bool s_last;
  Slice S = slice(A, blockIdx.y);
  if ((int)blockIdx.x >= S.nblk) return;
  const int64_t off = (int64_t)blockIdx.y * A.vstride;
  double dd = 0.0, aa = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S.n;
       i += (int64_t)S.nblk * blockDim.x) {
    const double d = a[off + i] - b[off + i];
    dd += d * d;
    aa += a[off + i] * a[off + i];
  }
  if (!grid_sum2(dd, aa, S.partials, &S.st->counter, sh, &s_last, S.nblk)) return;
  if (threadIdx.x == 0) {
    S.st->scratch0 = dd;
    S.st->scratch1 = aa;
  }
}

dim3 grid(const PcgArgs& a, int nrhs) { return dim3(pcg_blocks(a.n_kept), nrhs); }

// one grid for every slot of a batch: the largest any member would use
dim3 grid(const PcgBatch& b) {
  int g = 64;
  for (int i = 0; i < b.n; ++i) g = std::max(g, pcg_blocks(b.s[i].A.n_kept));
  return dim3(g, b.n);
}

}  // namespace

int launch_pcg_init(const mm_pointing_s* pt, const PcgArgs& a, int nrhs, double tol, int32_t max_iter,
                    int32_t fixed_iter, const OuterState* gate, hipStream_t s, bool from_x0) {
  hipLaunchKernelGGL(k_pcg_init, grid(a, nrhs), dim3(kPcgThreads), 0, s, a, pt->minv, tol, max_iter,
                     fixed_iter, gate, (int32_t)from_x0);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_pcg_iteration_tail(const mm_pointing_s* pt, const PcgArgs& a, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_alpha, grid(a, nrhs), dim3(kPcgThreads), 0, s, a);
  hipLaunchKernelGGL(k_pcg_update, grid(a, nrhs), dim3(kPcgThreads), 0, s, a, pt->minv);
  hipLaunchKernelGGL(k_pcg_direction, grid(a, nrhs), dim3(kPcgThreads), 0, s, a);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_diff_norm(const PcgArgs& a, int nrhs, const double* x, const double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_diff_norm, grid(a, nrhs), dim3(kPcgThreads), 0, s, a, x, y);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_init(const OuterArgs& o, const PcgArgs& a, int nrhs, hipStream_t s, bool from_x0) {
  hipLaunchKernelGGL(k_outer_init, grid(a, nrhs), dim3(kPcgThreads), 0, s, o, a, (int32_t)from_x0);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_add(const OuterArgs& o, const PcgArgs& a, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_add, grid(a, nrhs), dim3(kPcgThreads), 0, s, o, a);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_end(const OuterArgs& o, const PcgArgs& a, int nrhs, double tol, int32_t max_outer,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_outer_end, grid(a, nrhs), dim3(kPcgThreads), 0, s, o, a, tol, max_outer);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_pcg_iteration_tail_batch(const PcgBatch& b, hipStream_t s) {
  if (b.n == 0) return MM_OK;
  hipLaunchKernelGGL(k_pcg_alpha_b, grid(b), dim3(kPcgThreads), 0, s, b);
  hipLaunchKernelGGL(k_pcg_update_b, grid(b), dim3(kPcgThreads), 0, s, b);
  hipLaunchKernelGGL(k_pcg_direction_b, grid(b), dim3(kPcgThreads), 0, s, b);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_add_batch(const PcgBatch& b, hipStream_t s) {
  if (b.n == 0) return MM_OK;
  hipLaunchKernelGGL(k_outer_add_b, grid(b), dim3(kPcgThreads), 0, s, b);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_outer_end_batch(const PcgBatch& b, hipStream_t s) {
  if (b.n == 0) return MM_OK;
  hipLaunchKernelGGL(k_outer_end_b, grid(b), dim3(kPcgThreads), 0, s, b);
  hipLaunchKernelGGL(k_pcg_reinit_b, grid(b), dim3(kPcgThreads), 0, s, b);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
