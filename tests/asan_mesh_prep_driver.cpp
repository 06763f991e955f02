// Test driver: the host mesh preparation behind a C entry point, built with
// AddressSanitizer and UBSan by tests/test_host_sanitizers.py.
#include "mesh_prep.hpp"
extern "C" int asan_prep(int64_t n, const double* xy, int64_t e, const int32_t* tri, int64_t w, const int32_t* we,
                         double period, int reorder) {
  felbm::MeshPrep m;
  std::string err;
  int r = felbm::prepare_mesh(n, xy, e, tri, w, we, period, m, err, reorder != 0, 256);
  return r;
}
