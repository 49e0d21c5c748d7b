// Discrete adjoint of a taped rollout.
#include "qs_backward.h"

namespace qs {

hipError_t bwd_alloc(BwdBufs& bw, int N, int K, int H) {
  bw.N = N;
  bw.K = K;
  bw.H = H;
  return hipSuccess;
}

void bwd_free(BwdBufs& bw) {
  if (bw.seg) (void)hipFree(bw.seg);
  if (bw.lam) (void)hipFree(bw.lam);
  if (bw.gpart) (void)hipFree(bw.gpart);
  bw = BwdBufs{};
}

hipError_t run_backward(const DevCfg&, const SimBufs&, BwdBufs&, const float*, const float*, int,
                        int, const float*, const float*, float*, float*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace qs
