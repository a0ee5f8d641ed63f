// Instantiations of the forward-mode (Alg. 4) network kernels for width 16.
#include "mlp_fwd.h"

namespace pa {

int launch_mlp_fwd_h16(const PrepLayout& lay, int prec, const unsigned char* prep, int64_t n, const double* K,
                        double* out, int hess, hipStream_t s) {
  if (lay.L == 2 && lay.P == 3) return launch_mlp_t<16, 2, 3>(lay, prec, prep, n, K, out, hess, s);
  if (lay.L == 2 && lay.P == 5) return launch_mlp_t<16, 2, 5>(lay, prec, prep, n, K, out, hess, s);
  if (lay.L == 2 && lay.P == 9) return launch_mlp_t<16, 2, 9>(lay, prec, prep, n, K, out, hess, s);
  if (lay.L == 3 && lay.P == 3) return launch_mlp_t<16, 3, 3>(lay, prec, prep, n, K, out, hess, s);
  if (lay.L == 3 && lay.P == 5) return launch_mlp_t<16, 3, 5>(lay, prec, prep, n, K, out, hess, s);
  if (lay.L == 3 && lay.P == 9) return launch_mlp_t<16, 3, 9>(lay, prec, prep, n, K, out, hess, s);
  return -2;
}

}  // namespace pa
