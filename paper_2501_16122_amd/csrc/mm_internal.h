// Internal declarations shared by the HIP translation units of libmapmaker.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "mapmaker.h"

namespace mm {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define MM_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return mm::hip_fail(e_, #call); \
  } while (0)

// ---------------------------------------------------------------------------
// geometry of the timeline-domain work units
// ---------------------------------------------------------------------------

// A pointing tile: up to kTileSamples consecutive samples of one detector.
// kmin/kmax bound the compact pixel indices of its kept samples (kmax < kmin
// when it has none); the hot kernels bin into LDS slots k - kmin.
constexpr int kTileSamples = 4096;
struct PtTile {
  int64_t start;
  int32_t len;
  int32_t det;
  int32_t kmin;
  int32_t kmax;
};
static_assert(sizeof(PtTile) == 24, "PtTile layout");

// An overlap-save tile of the band-Toeplitz N^-1: it produces outputs
// [out_start, out_end) of one chunk [chunk_start, chunk_end) from the input
// window [out_start - (lambda - 1), out_start - (lambda - 1) + L).
struct FftTile {
  int64_t out_start;
  int64_t out_end;
  int64_t chunk_start;
  int64_t chunk_end;
  int32_t filter;
  int32_t wrap;  // 1: circulant chunk (window positions past its edges wrap around it)
};
static_assert(sizeof(FftTile) == 40, "FftTile layout");

// Halo-carrying tiles: consecutive tiles of one chunk start kCarryStride[a]
// samples apart, a multiple of the window positions one register element of
// every thread covers, so the gathered P x of a window's last elements is
// the next window's first, in the same registers.  A segment is
// a run of up to kSegTiles such tiles of one chunk, handled by one workgroup
// in order.
constexpr int64_t kCarryStride[2] = {8192, 24576};  // samples between carrying tiles (FP64, FP32 plan)
constexpr int kSegTiles = 64;  // longest segment
struct CarrySeg {
  int64_t first;  // index of its first tile in the halo-carrying tile list
  int32_t count;
  int32_t pad_;
};

// An interval of the template-filtered weight: samples [start, end) of one
// detector, with polynomial baselines of degree < order projected out.
constexpr int kMaxTplOrder = 8;
struct TplInterval {
  int64_t start;
  int64_t end;
  int32_t order;
  int32_t pad_;
};
static_assert(sizeof(TplInterval) == 24, "TplInterval layout");

// Real-signal length L and complex FFT length N = L/2 per arithmetic.
// FP64: L = 2^14 (8192 complex doubles = 128 KiB of LDS);
// FP32: L = 2^15 (16384 complex floats = 128 KiB of LDS).
constexpr int kFftN64 = 8192;
constexpr int kFftN32 = 16384;
// spectral-weight order of the two-per-CU half-buffer plans, FP64 and FP32:
// the number of region-major sequences of the four-step split, or 0 for the
// natural order of the Stockham passes (the FP64 plan: its four-step form
// spilled registers and ran slower)
constexpr int kHalfRegions[2] = {0, 32};
constexpr int kFftN32L = 32768;  // the longer FP32 plan
constexpr int kMaxLambda = 4096;

// Carves aligned sub-buffers out of one caller workspace.
struct Carver {
  char* base;
  size_t used = 0;
  size_t cap;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t n) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + n * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool fits() const { return used <= cap; }
};

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
}  // namespace mm

struct mm_pointing_s {
  int32_t dtype = MM_F64;
  int32_t ncomp = 3;  // values per pixel: 3 = I, Q, U; 2 = Q, U; 1 = I
  int64_t n_samples = 0;
  int32_t n_det = 0;
  int32_t n_pix = 0;
  int32_t n_kept = 0;
  int device = 0;
  const int32_t* pix = nullptr;
  const void* psi = nullptr;
  // optional precomputed (cos 2psi, sin 2psi) per sample, dtype pairs
  const void* weights = nullptr;
  std::vector<int64_t> det_offsets;
  std::vector<double> det_weight;
  // device state carved from the caller's workspace
  int32_t* hits = nullptr;       // [n_pix]
  uint8_t* mask = nullptr;       // [n_pix]
  int32_t* compact = nullptr;    // [n_pix]
  int32_t* kept = nullptr;       // [n_pix] (first n_kept used)
  double* blocks = nullptr;      // [nb * n_pix] upper triangles of P^T diag(N)^-1 P, nb = ncomp (ncomp + 1) / 2
  double* minv = nullptr;        // [nb * n_pix] upper triangles of the inverses (compact order)
  int32_t* sample_k = nullptr;   // [n_samples] compact index per sample, -1 = masked
  double* det_w = nullptr;       // [n_det]
  mm::PtTile* tiles = nullptr;   // [n_tiles]
  int64_t n_tiles = 0;
  int32_t* scan_tmp = nullptr;   // [n_scan_blocks + 1]
  int32_t* flags = nullptr;      // [4]: 0 = bad pixel seen, 1 = n_kept
};

struct mm_noise_s {
  // 0 = white, 1 = band-Toeplitz, 2 = circulant (band filter, periodic chunks),
  // 3 = white with polynomial templates marginalised per interval
  int kind = 0;
  int device = 0;
  // white (and the weights of the template-filtered form)
  int32_t n_det = 0;
  double* det_w = nullptr;
  // template-filtered: its intervals (partitioning the timeline; their
  // offsets are also kept in chunk_offsets for the detector checks)
  mm::TplInterval* tpl = nullptr;
  // band-Toeplitz
  int32_t lambda = 0;
  int32_t n_filt = 0;
  int64_t n_chunks = 0;
  std::vector<int64_t> chunk_offsets;
  std::vector<int32_t> chunk_filter;
  // per arithmetic (0 = FP64, 1 = FP32): tiles, spectral weights, twiddles
  mm::FftTile* tiles[2] = {nullptr, nullptr};
  int64_t n_tiles[2] = {0, 0};
  // halo-carrying tiles and their segments, per arithmetic
  mm::FftTile* ctiles[2] = {nullptr, nullptr};
  mm::CarrySeg* csegs[2] = {nullptr, nullptr};
  int64_t n_csegs[2] = {0, 0};
  void* ab[2] = {nullptr, nullptr};  // [n_filt][N] pairs (alpha_k, beta_k)
  // the same in the order of the two-per-CU half-buffer plans: region-major
  // (bin k1 + E k2 at k1 N/E + k2, E = kHalfRegions[a]) or, for E = 0, ab[a]
  void* abr[2] = {nullptr, nullptr};
  void* tw[2] = {nullptr, nullptr};  // [N] exp(-2 pi i k / N)
  // FP64 tables of the 16384-point plan (its tiles are the FP32 plan's);
  // its weights in region-major order: bin k1 + 16 k2 at k1 * 1024 + k2
  void* ab64l = nullptr;
  void* tw64l = nullptr;
  // the 32768-point FP32 plan: its tiles and FP32 tables (weights in
  // region-major order: bin k1 + 32 k2 at k1 * 1024 + k2)
  mm::FftTile* tiles32l = nullptr;
  int64_t n_tiles32l = 0;
  void* ab32l = nullptr;
  void* tw32l = nullptr;
  // operator variants picked by the autotuner, per problem shape
  struct Tuned {
    int64_t n_samples;
    int32_t n_kept, dtype, arith, nrhs, variant, ncomp;
  };
  mutable std::vector<Tuned> tuned;
};

namespace mm {

// Calls f.template operator()<NC>() with the map form's number of values
// per pixel as a compile-time constant.
template <class F>
int by_ncomp(int nc, F&& f) {
  switch (nc) {
    case 3: return f.template operator()<3>();
    case 2: return f.template operator()<2>();
    case 1: return f.template operator()<1>();
    default: return fail(MM_EINVAL, "map form must have 1, 2 or 3 values per pixel");
  }
}

// ---------------------------------------------------------------------------
// kernel launchers (each defined in the .hip file that holds its kernel)
// ---------------------------------------------------------------------------
int launch_pointing_build(mm_pointing_s* pt, int32_t min_hits, double cond_max, hipStream_t s);
int launch_compute_weights(const mm_pointing_s* pt, void* weights, hipStream_t s);
int launch_export(const mm_pointing_s* pt, int32_t* hits, uint8_t* mask, int32_t* compact,
                  int32_t* kept, double* minv, hipStream_t s);

// timeline-domain operators (white / diagonal parts)
int launch_apply_P(const mm_pointing_s* pt, const double* x, void* tod, int arith, hipStream_t s);
int launch_apply_PT(const mm_pointing_s* pt, const void* tod, double* q, int arith, hipStream_t s);
int launch_ninv_white(const mm_pointing_s* pt, const double* det_w, const void* in, void* out, int arith,
                      hipStream_t s);
// Right-hand-side batching of the fused operators: nrhs vectors at stride
// vstride (x and q), and per right-hand side a "done" flag at done[r *
// done_stride] (null: never done); a right-hand side whose flag is set is
// skipped.
struct RhsBatch {
  int32_t nrhs = 1;
  int64_t vstride = 0;
  const int32_t* done = nullptr;
  int32_t done_stride = 0;
};
// q += P^T diag(w) P x (q must hold the accumulation start, usually 0).
int launch_fused_white(const mm_pointing_s* pt, const double* det_w, const double* x, double* q, int arith,
                       const RhsBatch& rb, hipStream_t s);
// q += P^T diag(w) tod
int launch_rhs_white(const mm_pointing_s* pt, const double* det_w, const void* tod, double* q, int arith,
                     hipStream_t s);

// band-Toeplitz
int launch_ninv_toeplitz(const mm_pointing_s* pt, const mm_noise_s* nz, const void* in, void* out, int arith,
                         hipStream_t s);
// Variants of the fused band-Toeplitz operator (picked by the solver's
// autotuner): bit kOpLinearOrder takes tiles in launch order instead of the
// XCD-aware order; bit kOpNoStaging reads the map from global memory instead
// of staging the tile's pixel window in LDS.  Every variant computes the same
// sums (up to the order of floating-point atomics).
// Bit kOpCarry uses the halo-carrying tiles: a workgroup walks a segment of
// consecutive tiles and reuses the P x of the overlap instead of gathering
// it again (never staged; tile order as bit kOpLinearOrder says; only with
// stored pointing weights, else the plain tiles are used).
// Bit kOpHalfLds runs plain tiles with two workgroups per CU: the FFT
// exchanges go through half the LDS (real parts, then imaginary parts), so
// the memory phases of one tile overlap the FFT of another (tile order as
// bit kOpLinearOrder says; bits kOpNoStaging and kOpCarry do not apply).
// Bit kOpLongPlan runs plain tiles of the arithmetic's longer plan: in FP64
// 16384 points, the FP32 plan's tile length (75% of each window valid at
// lambda = 4096 instead of 50%); in FP32 32768 points (87.5% instead of
// 75%); one 1024-thread workgroup per CU with the exchanges through a half
// buffer (tile order as bit kOpLinearOrder says; the other bits do not
// apply).
constexpr int32_t kOpLinearOrder = 1, kOpNoStaging = 2, kOpCarry = 4, kOpHalfLds = 8, kOpLongPlan = 16,
                  kOpVariants = 32;
int launch_fused_toeplitz(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tod,
                          double* q, int arith, const RhsBatch& rb, hipStream_t s, int32_t variant = 0);
// template-filtered white weights (noise kind 3)
int launch_fused_templates(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tod,
                           double* q, int arith, const RhsBatch& rb, hipStream_t s);
int launch_ninv_templates(const mm_pointing_s* pt, const mm_noise_s* nz, const void* in, void* out, int arith,
                          hipStream_t s);
int prepare_toeplitz_tables(mm_noise_s* nz, const double* coeff_host, void* ws, size_t ws_bytes,
                            hipStream_t s, size_t* bytes_needed);

// operator helpers shared by the C entry points and the solver
int apply_A_impl(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, double* q, int arith,
                 const RhsBatch& rb, hipStream_t s, int32_t variant = 0);
int rhs_impl(const mm_pointing_s* pt, const mm_noise_s* nz, const void* tod, double* b, int arith, hipStream_t s);
int check_pointing(mm_pointing_t pt);
int check_noise_vs_pointing(const mm_noise_s* nz, const mm_pointing_s* pt);

// pixel domain
int launch_apply_M(const mm_pointing_s* pt, const double* r, double* z, hipStream_t s);
int launch_expand(const mm_pointing_s* pt, const double* x, double* full, hipStream_t s);
int launch_fill(double* p, int64_t n, double v, hipStream_t s);

// PCG
struct PcgState {
  double rho;
  double alpha;
  double beta;
  double bnorm;
  double rel;
  double tol;
  double scratch0;
  double scratch1;
  int32_t iter;
  int32_t done;
  int32_t breakdown;
  int32_t converged;
  int32_t max_iter;
  int32_t fixed_iter;
  uint32_t counter;
  int32_t pad_;
};
constexpr int kPcgBlocks = 256;   // largest grid of the vector kernels (partial sums per block)
// Grid of the vector kernels for a problem: fixed by its size, so its sums
// are deterministic (a batched launch spans the largest member's grid, and
// each member uses only its own count of blocks); larger grids spend more on the per-block partial sums
// than they gain in memory parallelism (64 blocks for small maps, 256 at
// 512^2 and beyond).
__host__ __device__ inline int pcg_blocks(int32_t n_kept) {
  const int g = n_kept / 1024;
  return g < 64 ? 64 : (g > kPcgBlocks ? kPcgBlocks : g);
}
constexpr int kPcgThreads = 256;
constexpr int32_t kPcgDoneStride = (int32_t)(sizeof(PcgState) / sizeof(int32_t));

// Vectors of nrhs right-hand sides at stride vstride; state/partials/history
// per right-hand side (kernels use blockIdx.y as the right-hand-side index).
struct PcgArgs {
  double *x, *r, *z, *p, *q;
  const double* b;
  double* partials;  // [nrhs][2 * kPcgBlocks]
  PcgState* st;      // [nrhs]
  double* hist;      // [nrhs][hist_len]
  int64_t vstride;
  int32_t n_kept;
  int32_t hist_len;
  int32_t ncomp;     // values per kept pixel (vectors hold ncomp * n_kept)
  int32_t max_iter;  // inner iteration cap of a re-initialised inner solve (batched refinement)
};

// Outer FP64 refinement state per right-hand side.
struct OuterState {
  double bnorm;
  double rel;
  double target;        // the outer tolerance, once the first outer step has ended (0 before)
  int32_t iters;        // outer steps taken
  int32_t inner_total;  // inner PCG iterations of finished inner solves
  int32_t converged;
  int32_t done;
  int32_t skip;         // 1: no outer step pending for this right-hand side
  int32_t breakdown;
  uint32_t counter;
  int32_t pad_;
};
constexpr int32_t kOuterSkipOffset = (int32_t)(offsetof(OuterState, skip) / sizeof(int32_t));
constexpr int32_t kOuterStride = (int32_t)(sizeof(OuterState) / sizeof(int32_t));

struct OuterArgs {
  double *xt, *rt;
  const double* b64;
  double* partials;  // [nrhs][2 * kPcgBlocks]
  OuterState* os;    // [nrhs]
  double* hist;      // [nrhs][hist_len]
  int64_t vstride;
  int32_t hist_len;
  int32_t max_outer;  // refinement step cap (batched refinement)
};

// ---------------------------------------------------------------------------
// Batched launches: up to kMaxBatch right-hand sides ("slots") of different
// solves advance in shared launches.  The slot tables travel by value as
// kernel arguments, so a batch needs no device memory of its own.
// ---------------------------------------------------------------------------
constexpr int kMaxBatch = 16;

// One slot of a batched operator launch: the fused A of one right-hand side.
struct OpSlot {
  const void* tiles;        // FftTile[] of the plan (band-Toeplitz), or the pointing's PtTile[]
  const void* ab;           // band-Toeplitz spectral weights of the plan
  const void* tw;           // band-Toeplitz twiddles of the plan
  const int32_t* sample_k;
  const void* psi;
  const void* wts;          // stored tangents tan psi, or null
  const double* det_w;      // white noise weights
  const double* x;
  double* q;
  const int32_t* done;      // the slot is skipped while *done != 0 (null: never)
  const void* iv;           // template intervals (TplInterval[])
  int64_t n_pt_tiles;       // template slots: pointing tiles (for the detector of an interval)
  int32_t lambda;
  int32_t wrap;             // band-Toeplitz: 1 for circulant chunks (their tiles wrap)
};
struct OpBatch {
  int32_t n = 0;
  int32_t pad_ = 0;
  int64_t off[kMaxBatch + 1] = {};  // slot s owns work items [off[s], off[s + 1])
  OpSlot s[kMaxBatch] = {};
};
static_assert(sizeof(OpBatch) <= 2048, "operator batch must stay a small kernel argument");

// q += P^T N^-1 P x for every slot, one persistent launch per noise kind.
// dtype / arith / weights / map form must be common to all slots of the launch.
int launch_toeplitz_batch(const OpBatch& b, int dtype, int arith, bool weights, int ncomp, hipStream_t s);
int launch_white_batch(const OpBatch& b, int dtype, int arith, int ncomp, hipStream_t s);
// weights: every slot has stored pointing weights usable in this arithmetic
int launch_templates_batch(const OpBatch& b, int dtype, int arith, bool weights, int ncomp, hipStream_t s);

// from_x0: start from the x already in place, with A x0 in q and
// ||b - A x0||^2, ||b||^2 in each state's scratch0/scratch1 (launch_diff_norm)
int launch_pcg_init(const mm_pointing_s* pt, const PcgArgs& a, int nrhs, double tol, int32_t max_iter,
                    int32_t fixed_iter, const OuterState* gate, hipStream_t s, bool from_x0 = false);
int launch_pcg_iteration_tail(const mm_pointing_s* pt, const PcgArgs& a, int nrhs, hipStream_t s);
// per right-hand side: st->scratch0 = ||x - y||^2, st->scratch1 = ||x||^2
int launch_diff_norm(const PcgArgs& a, int nrhs, const double* x, const double* y, hipStream_t s);
// from_x0: start from the xt already in place, with A64 xt in the inner q
int launch_outer_init(const OuterArgs& o, const PcgArgs& a, int nrhs, hipStream_t s, bool from_x0 = false);
int launch_outer_add(const OuterArgs& o, const PcgArgs& a, int nrhs, hipStream_t s);
int launch_outer_end(const OuterArgs& o, const PcgArgs& a, int nrhs, double tol, int32_t max_outer, hipStream_t s);

// One slot of a batched PCG launch: single right-hand-side views (slice 0)
// of a solver's inner and outer state, and its preconditioner blocks.
struct PcgSlot {
  PcgArgs A;          // A.max_iter: inner iteration cap
  OuterArgs O;        // O.max_outer: refinement step cap
  const double* minv;
  double tol;         // outer tolerance (mixed)
  double inner_tol;   // inner tolerance of a re-initialised inner solve
};
struct PcgBatch {
  int32_t n = 0;
  int32_t pad_ = 0;
  PcgSlot s[kMaxBatch] = {};
};
static_assert(sizeof(PcgBatch) <= 3072, "PCG batch must stay a small kernel argument");

int launch_pcg_iteration_tail_batch(const PcgBatch& b, hipStream_t s);
// the outer refinement step of every slot whose inner solve has ended:
// xt += x, q = 0 (then q += A64 xt by an operator launch), and
int launch_outer_add_batch(const PcgBatch& b, hipStream_t s);
// rt = b64 - q, the outer test, and the gated re-initialisation of the inner PCG
int launch_outer_end_batch(const PcgBatch& b, hipStream_t s);

}  // namespace mm
