// Checks of the C ABI's host-only paths: size queries (the band-Toeplitz
// tables' tile lists and the solver and pointing layouts are computed on the
// host), option defaults, argument validation and error paths.  None of
// these calls touches a GPU.  Built against the library's host code with
// AddressSanitizer and UndefinedBehaviorSanitizer: a sanitizer report or a
// failed check ends it with a non-zero status.
#include <cstdio>
#include <cstring>
#include <vector>

#include "mapmaker.h"

static int g_failures = 0;

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed (line %d): %s\n", __LINE__, #cond); \
      ++g_failures;                                                        \
    }                                                                      \
  } while (0)

int main() {
  CHECK(mm_abi_version() == 5);
  size_t sz = 0, sz2 = 0;

  // pointing workspace: both storage types, bad sizes and dtype refused
  CHECK(mm_pointing_workspace_size(1 << 20, 4, 4096, MM_F64, &sz) == MM_OK && sz > 0);
  CHECK(mm_pointing_workspace_size(1 << 20, 4, 4096, MM_F32, &sz2) == MM_OK && sz2 > 0 && sz2 <= sz);
  CHECK(mm_pointing_workspace_size(0, 1, 1, MM_F64, &sz) == MM_OK);
  CHECK(mm_pointing_workspace_size(-1, 4, 4096, MM_F64, &sz) == MM_EINVAL);
  CHECK(mm_pointing_workspace_size(100, 0, 4096, MM_F64, &sz) == MM_EINVAL);
  CHECK(mm_pointing_workspace_size(100, 1, 0, MM_F64, &sz) == MM_EINVAL);
  CHECK(mm_pointing_workspace_size(100, 1, 16, 7, &sz) == MM_EINVAL);
  CHECK(std::strlen(mm_last_error()) > 0);
  CHECK(mm_pointing_workspace_size(100, 1, 16, MM_F64, nullptr) == MM_EINVAL);

  // band-Toeplitz tables: ragged chunks at every band class, more filters
  // need more room; unordered chunks and bad bands refused
  std::vector<int64_t> off = {0, 300000, 700001, 1048576, 2000000, 2000000, 2100003};
  const int64_t n_ch = (int64_t)off.size() - 1;
  for (int lam : {1, 7, 64, 512, 4096}) {
    CHECK(mm_noise_toeplitz_workspace_size(lam, 1, off.data(), n_ch, &sz) == MM_OK && sz > 0);
    CHECK(mm_noise_toeplitz_workspace_size(lam, 3, off.data(), n_ch, &sz2) == MM_OK && sz2 > sz);
  }
  std::vector<int64_t> unordered = {0, 500, 400};
  CHECK(mm_noise_toeplitz_workspace_size(64, 1, unordered.data(), 2, &sz) == MM_EINVAL);
  CHECK(mm_noise_toeplitz_workspace_size(4097, 1, off.data(), n_ch, &sz) == MM_EINVAL);
  CHECK(mm_noise_toeplitz_workspace_size(0, 1, off.data(), n_ch, &sz) == MM_EINVAL);
  CHECK(mm_noise_toeplitz_workspace_size(64, 0, off.data(), n_ch, &sz) == MM_EINVAL);
  CHECK(mm_noise_toeplitz_workspace_size(64, 1, off.data(), n_ch, nullptr) == MM_EINVAL);
  CHECK(mm_noise_white_workspace_size(4, &sz) == MM_OK && sz == 4 * sizeof(double));
  CHECK(mm_noise_white_workspace_size(0, &sz) == MM_EINVAL);
  CHECK(mm_noise_templates_workspace_size(4, 100, &sz) == MM_OK && sz > 0);
  CHECK(mm_noise_templates_workspace_size(4, -1, &sz) == MM_EINVAL);

  // solver options and the workspace bound for every map form and precision
  mm_solve_opts o;
  CHECK(mm_solve_opts_default(&o) == MM_OK);
  CHECK(o.tol > 0.0 && o.max_iter > 0 && o.inner_tol > 0.0 && o.max_outer > 0);
  for (int nc = 1; nc <= 3; ++nc)
    for (int nrhs : {1, 4})
      for (int mixed : {0, 1}) {
        o.mixed = mixed;
        CHECK(mm_solver_workspace_bound(262144, nc, nrhs, &o, &sz) == MM_OK && sz > 0);
        CHECK(mm_solver_workspace_bound(1024, nc, nrhs, &o, &sz2) == MM_OK && sz2 < sz);
      }
  CHECK(mm_solver_workspace_bound(100, 4, 1, &o, &sz) == MM_EINVAL);
  CHECK(mm_solver_workspace_bound(100, 3, 0, &o, &sz) == MM_EINVAL);
  CHECK(mm_solver_workspace_bound(-1, 3, 1, &o, &sz) == MM_EINVAL);

  // the tuner's choice cache: round trip, replacement, malformed entries
  int32_t nt = -1;
  CHECK(mm_tune_cache_get(nullptr, 0, &nt) == MM_OK && nt == 0);
  mm_tune_entry te[2] = {{0, 28, MM_F64, MM_F64, 1, 3, 4096, 1, 16}, {0, 28, MM_F64, MM_F32, 1, 3, 4096, 1, 8}};
  CHECK(mm_tune_cache_put(te, 2) == MM_OK);
  mm_tune_entry back[4];
  CHECK(mm_tune_cache_get(back, 4, &nt) == MM_OK && nt == 2 && back[1].op_variant == 8);
  te[0].op_variant = 5;
  CHECK(mm_tune_cache_put(te, 1) == MM_OK);
  CHECK(mm_tune_cache_get(back, 1, &nt) == MM_OK && nt == 2 && back[0].op_variant == 5);
  te[1].op_variant = 32;
  CHECK(mm_tune_cache_put(te, 2) == MM_EINVAL);
  CHECK(mm_tune_cache_get(nullptr, 0, &nt) == MM_OK && nt == 2);
  CHECK(mm_tune_cache_get(nullptr, 1, &nt) == MM_EINVAL);
  CHECK(mm_tune_cache_put(nullptr, 1) == MM_EINVAL);

  // null handles and bad arguments are refused before any device work
  CHECK(mm_apply_A(nullptr, nullptr, nullptr, nullptr, MM_F64, nullptr) == MM_EINVAL);
  CHECK(mm_rhs(nullptr, nullptr, nullptr, nullptr, MM_F64, nullptr) == MM_EINVAL);
  CHECK(mm_solve_workspace_size(nullptr, nullptr, &o, &sz) == MM_EINVAL);
  CHECK(mm_solver_step(nullptr, 1) == MM_EINVAL);
  CHECK(mm_batch_step(nullptr, 1, 1) == MM_EINVAL);
  mm_noise_t nz = reinterpret_cast<mm_noise_t>(&g_failures);
  CHECK(mm_noise_toeplitz(nullptr, 64, 1, off.data(), nullptr, n_ch, nullptr, 0, nullptr, &nz) == MM_EINVAL &&
        nz == nullptr);
  CHECK(mm_pointing_destroy(nullptr) == MM_OK);
  CHECK(mm_noise_destroy(nullptr) == MM_OK);
  CHECK(mm_solver_destroy(nullptr) == MM_OK);

  if (g_failures) {
    std::fprintf(stderr, "%d checks failed\n", g_failures);
    return 1;
  }
  std::printf("host checks ok\n");
  return 0;
}
