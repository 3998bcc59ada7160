#include "hjpd_lintanh.hpp"

namespace hjpd {

struct LtState {
  int dummy;
};

int lt_create(LtState** out, const hjpd_desc&) {
  *out = nullptr;
  return hjpd_fail(HJPD_EUNSUPPORTED, "LINEAR_TANH not built yet");
}
void lt_destroy(LtState* s) { delete s; }
int lt_solve(LtState*, const hjpd_desc&, int64_t, const void*, const void*, const int32_t*, const void*, const void*,
             void*, void*, void*, int32_t*, int32_t*, hipStream_t, hipEvent_t, hipEvent_t, int*, bool*) {
  return hjpd_fail(HJPD_EUNSUPPORTED, "LINEAR_TANH not built yet");
}
int lt_value_grad(LtState*, const hjpd_desc&, int64_t, const void*, const void*, const int32_t*, const void*,
                  const void*, const void*, int, int, void*, void*, void*, void*, hipStream_t) {
  return hjpd_fail(HJPD_EUNSUPPORTED, "LINEAR_TANH not built yet");
}

}  // namespace hjpd
