// yy_pair_mfma.hip -- pairwise kernel on the matrix cores (placeholder).
#include "yy_internal.h"

namespace yy {

yy_status launch_pair_mfma(hipStream_t, const PairArgs&, int) {
  return fail(YY_ERR_UNSUPPORTED, "matrix-core pairwise kernel not built");
}

}  // namespace yy
