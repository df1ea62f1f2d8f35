// C entry points around the host levels of the forward-model search, for
// tests/test_mlp_host.py (built together with csrc/mlp_host.cpp).
#include "../../paper_2107_01715_amd/csrc/mlp_host.h"

extern "C" {
void* shim_create(int A, const float* dev_blob) {
  auto* m = new bcts::MlpHost();
  bcts::mlp_host_prepare(*m, A, dev_blob);
  return m;
}
void shim_level(void* m, long long n, const float* ps, const float* pret, float gpow, float* os, float* oret,
                float* ov) {
  bcts::mlp_host_level(*static_cast<bcts::MlpHost*>(m), n, ps, pret, gpow, os, oret, ov);
}
void shim_free(void* m) { delete static_cast<bcts::MlpHost*>(m); }
}
