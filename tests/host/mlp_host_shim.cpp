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
void shim_search(void* m, int n, const float* states, int d, float gamma, int corr, float pen_e, float pen_o,
                 float scale, int32_t* act, float* q) {
  bcts::mlp_host_search(*static_cast<bcts::MlpHost*>(m), n, states, d, gamma, corr != 0, pen_e, pen_o, scale, act, q);
}
void shim_free(void* m) { delete static_cast<bcts::MlpHost*>(m); }
}
