// C ABI of libmapmaker: argument checking, workspace carving and the host
// side of the PCG solve.  Every step of the computation runs in the HIP
// kernels of the other translation units; this file only enqueues them.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "mm_internal.h"

namespace mm {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
  return MM_EHIP;
}

namespace {

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool valid_dtype(int d) { return d == MM_F64 || d == MM_F32; }

// Workspace layout of a pointing handle (also used for the size query).
struct PtLayout {
  int32_t* hits;
  uint8_t* mask;
  int32_t* compact;
  int32_t* kept;
  double* blocks;
  double* minv;
  int32_t* sample_k;
  double* det_w;
  PtTile* tiles;
  int32_t* scan_tmp;
  int32_t* flags;
};

int64_t count_tiles(const int64_t* offs, int32_t n_det) {
  int64_t n = 0;
  for (int32_t d = 0; d < n_det; ++d) n += (offs[d + 1] - offs[d] + kTileSamples - 1) / kTileSamples;
  return n;
}

size_t carve_pointing(Carver& cv, int64_t n_samples, int32_t n_det, int32_t n_pix, int64_t n_tiles, PtLayout* L) {
  const int64_t nb_scan = (n_pix + 1023) / 1024;
  L->hits = cv.take<int32_t>(n_pix);
  L->mask = cv.take<uint8_t>(n_pix);
  L->compact = cv.take<int32_t>(n_pix);
  L->kept = cv.take<int32_t>(n_pix);
  L->blocks = cv.take<double>(6 * (size_t)n_pix);
  L->minv = cv.take<double>(6 * (size_t)n_pix);
  L->sample_k = cv.take<int32_t>(n_samples);
  L->det_w = cv.take<double>(n_det);
  L->tiles = cv.take<PtTile>(n_tiles);
  L->scan_tmp = cv.take<int32_t>(nb_scan + 1);
  L->flags = cv.take<int32_t>(4);
  return cv.used;
}

}  // namespace

int apply_A_impl(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, double* q, int arith,
                 const RhsBatch& rb, hipStream_t s, int32_t variant) {
  if (nz->kind == 0) return launch_fused_white(pt, nz->det_w, x, q, arith, rb, s);
  if (nz->kind == 3) return launch_fused_templates(pt, nz, x, nullptr, q, arith, rb, s);
  return launch_fused_toeplitz(pt, nz, x, nullptr, q, arith, rb, s, variant);
}

int rhs_impl(const mm_pointing_s* pt, const mm_noise_s* nz, const void* tod, double* b, int arith, hipStream_t s) {
  int rc = launch_fill(b, (int64_t)pt->ncomp * pt->n_kept, 0.0, s);
  if (rc) return rc;
  if (nz->kind == 0) return launch_rhs_white(pt, nz->det_w, tod, b, arith, s);
  if (nz->kind == 3) return launch_fused_templates(pt, nz, nullptr, tod, b, arith, RhsBatch{}, s);
  return launch_fused_toeplitz(pt, nz, nullptr, tod, b, arith, RhsBatch{}, s);
}

int check_pointing(mm_pointing_t pt) {
  if (pt == nullptr) return fail(MM_EINVAL, "null pointing handle");
  return MM_OK;
}

int check_noise_vs_pointing(const mm_noise_s* nz, const mm_pointing_s* pt) {
  if (nz == nullptr) return fail(MM_EINVAL, "null noise handle");
  if (nz->kind == 0) {
    if (nz->n_det != pt->n_det) return fail(MM_EINVAL, "white noise has a different detector count");
    return MM_OK;
  }
  if (nz->kind == 3) {
    if (nz->n_det != pt->n_det) return fail(MM_EINVAL, "template weights have a different detector count");
    if (nz->chunk_offsets.back() != pt->n_samples)
      return fail(MM_EINVAL, "template intervals must end at the last sample of the timeline");
  }
  if (nz->chunk_offsets.back() > pt->n_samples) return fail(MM_EINVAL, "noise chunks extend past the timeline");
  // no chunk may straddle a detector start
  size_t d = 1;
  for (int64_t c = 0; c < nz->n_chunks; ++c) {
    const int64_t a = nz->chunk_offsets[c], b = nz->chunk_offsets[c + 1];
    while (d < pt->det_offsets.size() && pt->det_offsets[d] <= a) ++d;
    if (d < pt->det_offsets.size() && pt->det_offsets[d] < b)
      return fail(MM_EINVAL, "a noise chunk crosses a detector start");
  }
  return MM_OK;
}

int check_chunks(const int64_t* offs, int64_t n_chunks) {
  if (!offs || n_chunks < 0) return fail(MM_EINVAL, "bad chunk offsets");
  if (offs[0] < 0) return fail(MM_EINVAL, "chunk offsets must be >= 0");
  for (int64_t c = 0; c < n_chunks; ++c)
    if (offs[c + 1] < offs[c]) return fail(MM_EINVAL, "chunk offsets must be non-decreasing");
  return MM_OK;
}

int make_banded_noise(int kind, const double* coeff_host, int32_t lambda, int32_t n_filt,
                      const int64_t* chunk_offsets_host, const int32_t* chunk_filter_host, int64_t n_chunks,
                      void* workspace, size_t ws_bytes, void* stream, mm_noise_t* out) {
  if (!out) return fail(MM_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (!coeff_host || !workspace || lambda < 1 || lambda > kMaxLambda || n_filt < 1)
    return fail(MM_EINVAL, "bad Toeplitz arguments (1 <= lambda <= 4096)");
  if (int rc = check_chunks(chunk_offsets_host, n_chunks)) return rc;
  for (int64_t i = 0; i < (int64_t)n_filt * lambda; ++i)
    if (!std::isfinite(coeff_host[i])) return fail(MM_EINVAL, "non-finite Toeplitz coefficient");
  auto* nz = new (std::nothrow) mm_noise_s();
  if (!nz) return fail(MM_EINVAL, "out of host memory");
  nz->kind = kind;
  nz->lambda = lambda;
  nz->n_filt = n_filt;
  nz->n_chunks = n_chunks;
  nz->chunk_offsets.assign(chunk_offsets_host, chunk_offsets_host + n_chunks + 1);
  nz->chunk_filter.resize(n_chunks);
  for (int64_t c = 0; c < n_chunks; ++c) {
    const int32_t f = chunk_filter_host ? chunk_filter_host[c] : 0;
    if (f < 0 || f >= n_filt) {
      delete nz;
      return fail(MM_EINVAL, "chunk_filter out of range");
    }
    nz->chunk_filter[c] = f;
  }
  (void)hipGetDevice(&nz->device);
  int rc = prepare_toeplitz_tables(nz, coeff_host, workspace, ws_bytes, as_stream(stream), nullptr);
  if (rc) {
    delete nz;
    return rc;
  }
  *out = nz;
  return MM_OK;
}

}  // namespace mm

using namespace mm;

extern "C" {

const char* mm_last_error(void) { return g_last_error.c_str(); }

int mm_abi_version(void) { return 5; }

int mm_pointing_workspace_size(int64_t n_samples, int32_t n_det, int32_t n_pix, int32_t dtype, size_t* bytes) {
  if (!bytes || n_samples < 0 || n_det <= 0 || n_pix <= 0) return fail(MM_EINVAL, "bad pointing sizes");
  if (!valid_dtype(dtype)) return fail(MM_EINVAL, "dtype must be MM_F64 or MM_F32");
  // worst case tile count: every detector may add one partial tile
  const int64_t n_tiles = n_samples / kTileSamples + n_det;
  Carver cv(nullptr, 0);
  PtLayout L;
  *bytes = carve_pointing(cv, n_samples, n_det, n_pix, n_tiles, &L);
  return MM_OK;
}

int mm_pointing_build(const int32_t* pix, const void* psi, int32_t dtype, int64_t n_samples,
                      const int64_t* det_offsets_host, int32_t n_det, const double* det_weight_host, int32_t n_pix,
                      int32_t min_hits, double cond_max, void* workspace, size_t ws_bytes, void* stream,
                      mm_pointing_t* out) {
  return mm_pointing_build_stokes(pix, psi, dtype, n_samples, det_offsets_host, n_det, det_weight_host, n_pix,
                                  MM_STOKES_IQU, min_hits, cond_max, workspace, ws_bytes, stream, out);
}

int mm_pointing_build_stokes(const int32_t* pix, const void* psi, int32_t dtype, int64_t n_samples,
                             const int64_t* det_offsets_host, int32_t n_det, const double* det_weight_host,
                             int32_t n_pix, int32_t stokes, int32_t min_hits, double cond_max, void* workspace,
                             size_t ws_bytes, void* stream, mm_pointing_t* out) {
  if (!out) return fail(MM_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (!valid_dtype(dtype)) return fail(MM_EINVAL, "dtype must be MM_F64 or MM_F32");
  if (stokes != MM_STOKES_IQU && stokes != MM_STOKES_QU && stokes != MM_STOKES_I)
    return fail(MM_EINVAL, "stokes must be MM_STOKES_IQU, MM_STOKES_QU or MM_STOKES_I");
  if (n_samples < 0 || n_det <= 0 || n_pix <= 0) return fail(MM_EINVAL, "bad sizes");
  if (n_samples > 0 && !pix) return fail(MM_EINVAL, "null pix");
  if (n_samples > 0 && !psi && stokes != MM_STOKES_I) return fail(MM_EINVAL, "null psi (needed unless stokes = I)");
  if (!det_offsets_host || !det_weight_host || !workspace) return fail(MM_EINVAL, "null argument");
  if (det_offsets_host[0] != 0 || det_offsets_host[n_det] != n_samples)
    return fail(MM_EINVAL, "det_offsets must start at 0 and end at n_samples");
  for (int32_t d = 0; d < n_det; ++d) {
    if (det_offsets_host[d + 1] < det_offsets_host[d]) return fail(MM_EINVAL, "det_offsets must be non-decreasing");
    if (!(det_weight_host[d] >= 0.0) || !std::isfinite(det_weight_host[d]))
      return fail(MM_EINVAL, "detector weights must be finite and >= 0");
  }
  size_t need = 0;
  mm_pointing_workspace_size(n_samples, n_det, n_pix, dtype, &need);
  if (ws_bytes < need) return fail(MM_ENOSPC, "pointing workspace too small");
  hipStream_t s = as_stream(stream);

  auto* pt = new (std::nothrow) mm_pointing_s();
  if (!pt) return fail(MM_EINVAL, "out of host memory");
  pt->dtype = dtype;
  pt->ncomp = stokes;
  pt->n_samples = n_samples;
  pt->n_det = n_det;
  pt->n_pix = n_pix;
  pt->pix = pix;
  pt->psi = stokes == MM_STOKES_I ? nullptr : psi;  // the intensity-only row never uses the angle
  pt->det_offsets.assign(det_offsets_host, det_offsets_host + n_det + 1);
  pt->det_weight.assign(det_weight_host, det_weight_host + n_det);
  (void)hipGetDevice(&pt->device);

  std::vector<PtTile> tiles;
  for (int32_t d = 0; d < n_det; ++d)
    for (int64_t t = det_offsets_host[d]; t < det_offsets_host[d + 1]; t += kTileSamples) {
      const int64_t len = std::min<int64_t>(kTileSamples, det_offsets_host[d + 1] - t);
      tiles.push_back(PtTile{t, (int32_t)len, d, 0, -1});
    }
  pt->n_tiles = (int64_t)tiles.size();
  Carver cv(workspace, ws_bytes);
  PtLayout L;
  carve_pointing(cv, n_samples, n_det, n_pix, pt->n_tiles, &L);
  pt->hits = L.hits;
  pt->mask = L.mask;
  pt->compact = L.compact;
  pt->kept = L.kept;
  pt->blocks = L.blocks;
  pt->minv = L.minv;
  pt->sample_k = L.sample_k;
  pt->det_w = L.det_w;
  pt->tiles = L.tiles;
  pt->scan_tmp = L.scan_tmp;
  pt->flags = L.flags;

  auto bail = [&](int rc) {
    delete pt;
    return rc;
  };
  hipError_t e;
  if (!tiles.empty() &&
      (e = hipMemcpyAsync(pt->tiles, tiles.data(), tiles.size() * sizeof(PtTile), hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return bail(hip_fail(e, "upload tiles"));
  if ((e = hipMemcpyAsync(pt->det_w, det_weight_host, sizeof(double) * n_det, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return bail(hip_fail(e, "upload weights"));
  int rc = launch_pointing_build(pt, min_hits, cond_max, s);
  if (rc) return bail(rc);
  int32_t flags[2] = {0, 0};
  if ((e = hipMemcpyAsync(flags, pt->flags, sizeof(flags), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return bail(hip_fail(e, "read build flags"));
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "build sync"));
  if (flags[0] & 1) return bail(fail(MM_EINVAL, "pixel index outside [0, n_pix)"));
  if (flags[0] & 2) return bail(fail(MM_EINVAL, "psi not finite or |2 psi| >= 4e8"));
  pt->n_kept = flags[1];
  *out = pt;
  return MM_OK;
}

int mm_pointing_info(mm_pointing_t pt, int32_t* n_kept, int64_t* n_samples, int32_t* n_pix, int32_t* n_det,
                     int32_t* dtype) {
  if (int rc = check_pointing(pt)) return rc;
  if (n_kept) *n_kept = pt->n_kept;
  if (n_samples) *n_samples = pt->n_samples;
  if (n_pix) *n_pix = pt->n_pix;
  if (n_det) *n_det = pt->n_det;
  if (dtype) *dtype = pt->dtype;
  return MM_OK;
}

int mm_pointing_stokes(mm_pointing_t pt, int32_t* stokes) {
  if (int rc = check_pointing(pt)) return rc;
  if (!stokes) return fail(MM_EINVAL, "null output");
  *stokes = pt->ncomp;
  return MM_OK;
}

int mm_pointing_export(mm_pointing_t pt, int32_t* hits, uint8_t* mask, int32_t* compact, int32_t* kept, double* minv,
                       void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  return launch_export(pt, hits, mask, compact, kept, minv, as_stream(stream));
}

int mm_pointing_attach_weights(mm_pointing_t pt, void* weights, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (weights == nullptr) {
    pt->weights = nullptr;
    return MM_OK;
  }
  if (pt->ncomp == 1) return fail(MM_EINVAL, "the intensity-only form has no pointing weights");
  if (int rc = launch_compute_weights(pt, weights, as_stream(stream))) return rc;
  pt->weights = weights;
  return MM_OK;
}

int mm_pointing_destroy(mm_pointing_t pt) {
  delete pt;
  return MM_OK;
}

int mm_noise_white_workspace_size(int32_t n_det, size_t* bytes) {
  if (!bytes || n_det <= 0) return fail(MM_EINVAL, "bad n_det");
  *bytes = sizeof(double) * (size_t)n_det;
  return MM_OK;
}

int mm_noise_templates_workspace_size(int32_t n_det, int64_t n_intervals, size_t* bytes) {
  if (!bytes || n_det <= 0 || n_intervals < 0) return fail(MM_EINVAL, "bad template sizes");
  Carver cv(nullptr, 0);
  cv.take<double>(n_det);
  cv.take<TplInterval>(n_intervals);
  *bytes = cv.used;
  return MM_OK;
}

int mm_noise_templates(const double* det_weight_host, int32_t n_det, const int64_t* interval_offsets_host,
                       const int32_t* interval_order_host, int32_t order, int64_t n_intervals, void* workspace,
                       size_t ws_bytes, void* stream, mm_noise_t* out) {
  if (!out) return fail(MM_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (!det_weight_host || n_det <= 0 || !workspace || !interval_offsets_host || n_intervals < 0)
    return fail(MM_EINVAL, "bad template arguments");
  for (int32_t d = 0; d < n_det; ++d)
    if (!(det_weight_host[d] >= 0.0) || !std::isfinite(det_weight_host[d]))
      return fail(MM_EINVAL, "detector weights must be finite and >= 0");
  if (interval_offsets_host[0] != 0) return fail(MM_EINVAL, "template intervals must start at sample 0");
  if (int rc = check_chunks(interval_offsets_host, n_intervals)) return rc;
  std::vector<TplInterval> iv(n_intervals);
  for (int64_t i = 0; i < n_intervals; ++i) {
    const int32_t o = interval_order_host ? interval_order_host[i] : order;
    if (o < 0 || o > kMaxTplOrder) return fail(MM_EINVAL, "template order must be in [0, 8]");
    iv[i] = TplInterval{interval_offsets_host[i], interval_offsets_host[i + 1], o, 0};
  }
  size_t need = 0;
  mm_noise_templates_workspace_size(n_det, n_intervals, &need);
  if (ws_bytes < need) return fail(MM_ENOSPC, "noise workspace too small");
  auto* nz = new (std::nothrow) mm_noise_s();
  if (!nz) return fail(MM_EINVAL, "out of host memory");
  nz->kind = 3;
  nz->n_det = n_det;
  nz->n_chunks = n_intervals;
  nz->chunk_offsets.assign(interval_offsets_host, interval_offsets_host + n_intervals + 1);
  Carver cv(workspace, ws_bytes);
  nz->det_w = cv.take<double>(n_det);
  nz->tpl = cv.take<TplInterval>(n_intervals);
  (void)hipGetDevice(&nz->device);
  hipStream_t s = as_stream(stream);
  hipError_t e = hipMemcpyAsync(nz->det_w, det_weight_host, sizeof(double) * n_det, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n_intervals > 0)
    e = hipMemcpyAsync(nz->tpl, iv.data(), sizeof(TplInterval) * n_intervals, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete nz;
    return hip_fail(e, "upload template tables");
  }
  *out = nz;
  return MM_OK;
}

int mm_noise_white(const double* det_weight_host, int32_t n_det, void* workspace, size_t ws_bytes, void* stream,
                   mm_noise_t* out) {
  if (!out) return fail(MM_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (!det_weight_host || n_det <= 0 || !workspace) return fail(MM_EINVAL, "bad white-noise arguments");
  if (ws_bytes < sizeof(double) * (size_t)n_det) return fail(MM_ENOSPC, "noise workspace too small");
  for (int32_t d = 0; d < n_det; ++d)
    if (!(det_weight_host[d] >= 0.0) || !std::isfinite(det_weight_host[d]))
      return fail(MM_EINVAL, "detector weights must be finite and >= 0");
  auto* nz = new (std::nothrow) mm_noise_s();
  if (!nz) return fail(MM_EINVAL, "out of host memory");
  nz->kind = 0;
  nz->n_det = n_det;
  nz->det_w = static_cast<double*>(workspace);
  (void)hipGetDevice(&nz->device);
  hipError_t e = hipMemcpyAsync(nz->det_w, det_weight_host, sizeof(double) * n_det, hipMemcpyHostToDevice,
                                as_stream(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
  if (e != hipSuccess) {
    delete nz;
    return hip_fail(e, "upload white-noise weights");
  }
  *out = nz;
  return MM_OK;
}


int mm_noise_toeplitz_workspace_size(int32_t lambda, int32_t n_filt, const int64_t* chunk_offsets_host,
                                     int64_t n_chunks, size_t* bytes) {
  if (!bytes || lambda < 1 || lambda > kMaxLambda || n_filt < 1) return fail(MM_EINVAL, "bad Toeplitz sizes");
  if (int rc = check_chunks(chunk_offsets_host, n_chunks)) return rc;
  mm_noise_s tmp;
  tmp.kind = 1;
  tmp.lambda = lambda;
  tmp.n_filt = n_filt;
  tmp.n_chunks = n_chunks;
  tmp.chunk_offsets.assign(chunk_offsets_host, chunk_offsets_host + n_chunks + 1);
  tmp.chunk_filter.assign(n_chunks, 0);
  return prepare_toeplitz_tables(&tmp, nullptr, nullptr, 0, nullptr, bytes);
}


int mm_noise_toeplitz(const double* coeff_host, int32_t lambda, int32_t n_filt, const int64_t* chunk_offsets_host,
                      const int32_t* chunk_filter_host, int64_t n_chunks, void* workspace, size_t ws_bytes,
                      void* stream, mm_noise_t* out) {
  return make_banded_noise(1, coeff_host, lambda, n_filt, chunk_offsets_host, chunk_filter_host, n_chunks, workspace,
                           ws_bytes, stream, out);
}

int mm_noise_circulant(const double* coeff_host, int32_t lambda, int32_t n_filt, const int64_t* chunk_offsets_host,
                       const int32_t* chunk_filter_host, int64_t n_chunks, void* workspace, size_t ws_bytes,
                       void* stream, mm_noise_t* out) {
  if (!out) return fail(MM_EINVAL, "null output handle pointer");
  *out = nullptr;
  if (chunk_offsets_host && lambda >= 1)
    for (int64_t c = 0; c < n_chunks; ++c) {
      const int64_t n = chunk_offsets_host[c + 1] - chunk_offsets_host[c];
      if (n > 0 && n <= 2 * (int64_t)(lambda - 1))
        return fail(MM_EINVAL, "a circulant chunk must be longer than 2 (lambda - 1)");
    }
  return make_banded_noise(2, coeff_host, lambda, n_filt, chunk_offsets_host, chunk_filter_host, n_chunks, workspace,
                           ws_bytes, stream, out);
}


int mm_noise_destroy(mm_noise_t nz) {
  delete nz;
  return MM_OK;
}

int mm_apply_P(mm_pointing_t pt, const double* x, void* tod, int32_t arith, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (!valid_dtype(arith)) return fail(MM_EINVAL, "bad arith");
  if ((pt->n_kept && !x) || (pt->n_samples && !tod)) return fail(MM_EINVAL, "null vector");
  return launch_apply_P(pt, x, tod, arith, as_stream(stream));
}

int mm_apply_PT(mm_pointing_t pt, const void* tod, double* q, int32_t arith, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (!valid_dtype(arith)) return fail(MM_EINVAL, "bad arith");
  if ((pt->n_kept && !q) || (pt->n_samples && !tod)) return fail(MM_EINVAL, "null vector");
  hipStream_t s = as_stream(stream);
  if (int rc = launch_fill(q, (int64_t)pt->ncomp * pt->n_kept, 0.0, s)) return rc;
  return launch_apply_PT(pt, tod, q, arith, s);
}

int mm_apply_Ninv(mm_noise_t nz, mm_pointing_t pt, const void* tod_in, void* tod_out, int32_t arith, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
  if (!valid_dtype(arith)) return fail(MM_EINVAL, "bad arith");
  if (pt->n_samples && (!tod_in || !tod_out)) return fail(MM_EINVAL, "null timeline");
  if (tod_in == tod_out && pt->n_samples) return fail(MM_EINVAL, "tod_out must not alias tod_in");
  hipStream_t s = as_stream(stream);
  if (nz->kind == 0) return launch_ninv_white(pt, nz->det_w, tod_in, tod_out, arith, s);
  if (nz->kind == 3) return launch_ninv_templates(pt, nz, tod_in, tod_out, arith, s);
  // samples outside every chunk are zero
  const size_t esz = pt->dtype == MM_F64 ? 8 : 4;
  MM_HIP(hipMemsetAsync(tod_out, 0, esz * (size_t)pt->n_samples, s));
  return launch_ninv_toeplitz(pt, nz, tod_in, tod_out, arith, s);
}

int mm_apply_A(mm_pointing_t pt, mm_noise_t nz, const double* x, double* q, int32_t arith, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
  if (!valid_dtype(arith)) return fail(MM_EINVAL, "bad arith");
  if (pt->n_kept && (!x || !q)) return fail(MM_EINVAL, "null vector");
  hipStream_t s = as_stream(stream);
  if (int rc = launch_fill(q, (int64_t)pt->ncomp * pt->n_kept, 0.0, s)) return rc;
  return apply_A_impl(pt, nz, x, q, arith, RhsBatch{}, s);
}

int mm_apply_A_variant(mm_pointing_t pt, mm_noise_t nz, const double* x, double* q, int32_t arith, int32_t variant,
                       void* stream) {
  if (variant < 0 || variant >= kOpVariants) return fail(MM_EINVAL, "operator variant out of range");
  if (int rc = check_pointing(pt)) return rc;
  if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
  if (!valid_dtype(arith)) return fail(MM_EINVAL, "bad arith");
  if (pt->n_kept && (!x || !q)) return fail(MM_EINVAL, "null vector");
  hipStream_t s = as_stream(stream);
  if (int rc = launch_fill(q, (int64_t)pt->ncomp * pt->n_kept, 0.0, s)) return rc;
  return apply_A_impl(pt, nz, x, q, arith, RhsBatch{}, s, variant);
}

int mm_apply_A_multi(mm_pointing_t pt, mm_noise_t nz, int32_t n_rhs, const double* x, double* q, int32_t arith,
                     void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
  if (!valid_dtype(arith) || n_rhs < 1) return fail(MM_EINVAL, "bad arith or n_rhs");
  if (pt->n_kept && (!x || !q)) return fail(MM_EINVAL, "null vector");
  hipStream_t s = as_stream(stream);
  const int64_t n3 = (int64_t)pt->ncomp * pt->n_kept;
  if (int rc = launch_fill(q, n3 * n_rhs, 0.0, s)) return rc;
  RhsBatch rb;
  rb.nrhs = n_rhs;
  rb.vstride = n3;
  return apply_A_impl(pt, nz, x, q, arith, rb, s);
}

int mm_rhs(mm_pointing_t pt, mm_noise_t nz, const void* tod, double* b, int32_t arith, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (int rc = check_noise_vs_pointing(nz, pt)) return rc;
  if (!valid_dtype(arith)) return fail(MM_EINVAL, "bad arith");
  if ((pt->n_kept && !b) || (pt->n_samples && !tod)) return fail(MM_EINVAL, "null vector");
  return rhs_impl(pt, nz, tod, b, arith, as_stream(stream));
}

int mm_apply_M(mm_pointing_t pt, const double* r, double* z, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (pt->n_kept && (!r || !z)) return fail(MM_EINVAL, "null vector");
  return launch_apply_M(pt, r, z, as_stream(stream));
}

int mm_expand_map(mm_pointing_t pt, const double* x, double* map_full, void* stream) {
  if (int rc = check_pointing(pt)) return rc;
  if (!map_full || (pt->n_kept && !x)) return fail(MM_EINVAL, "null vector");
  return launch_expand(pt, x, map_full, as_stream(stream));
}

}  // extern "C"
