// Host sanitizer run of the library's host code (test infrastructure): built
// by tests/test_host_sanitizers.py with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only, it runs the host-only
// entry points (the hierarchy builders and their checks on random,
// degenerate and collinear triangle sets, the information-word packing, the
// store size) and, with no GPU present, the error return of pv_create.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "pv.h"

static bool check(const std::vector<float>& v, uint32_t n, const char* what) {
  for (int32_t kind = 0; kind < 2; ++kind) {
    uint32_t out[4] = {0, 0, 0, 0};
    if (pv_hierarchy_info(v.data(), n, kind, out) != PV_OK || out[3] != 1) {
      std::printf("hierarchy check failed: %s, n %u, kind %d\n", what, n, kind);
      return false;
    }
  }
  return true;
}

int main() {
  std::mt19937 rng(5);
  std::uniform_real_distribution<float> U(-1.0f, 1.0f);
  for (uint32_t n : {1u, 2u, 3u, 7u, 9u, 64u, 1000u, 20000u}) {
    std::vector<float> v(9 * (size_t)n);
    for (auto& x : v) x = U(rng);
    if (!check(v, n, "random")) return 1;
  }
  {  // every triangle the same (equal centroids, equal boxes)
    const uint32_t n = 5000;
    std::vector<float> v(9 * (size_t)n);
    for (uint32_t i = 0; i < n; ++i)
      for (int k = 0; k < 9; ++k) v[9 * (size_t)i + k] = 0.1f * (float)k;
    if (!check(v, n, "identical")) return 1;
  }
  {  // zero-area triangles along a line
    const uint32_t n = 3000;
    std::vector<float> v(9 * (size_t)n);
    for (uint32_t i = 0; i < n; ++i)
      for (int k = 0; k < 3; ++k) {
        const float t = (float)i / n + 1e-4f * (float)k;
        v[9 * (size_t)i + 3 * k + 0] = t;
        v[9 * (size_t)i + 3 * k + 1] = 2.0f * t;
        v[9 * (size_t)i + 3 * k + 2] = -t;
      }
    if (!check(v, n, "collinear")) return 1;
  }
  uint32_t out[4];
  if (pv_hierarchy_info(nullptr, 3, 0, out) != PV_ERR_ARG) return 2;
  for (uint32_t w : {0u, 1u, 0x3fffffu, 0xffffffffu}) {
    uint32_t c, n, s, r, u;
    pv_info_unpack(w, &c, &n, &s, &r, &u);
    if (pv_info_pack(c, n, s, r, u) != w) return 3;
  }
  if (pv_store_bytes(3000000, 7) != 3000000ull * (32ull * 7 + 16ull)) return 4;
  // without a GPU the context cannot be created: an error, no context
  pv_ctx* ctx = nullptr;
  const pv_status st = pv_create(&ctx, nullptr);
  if (st == PV_OK) {
    pv_destroy(ctx);
  } else if (ctx != nullptr) {
    return 5;
  }
  std::printf("sanitized host run done\n");
  return 0;
}
