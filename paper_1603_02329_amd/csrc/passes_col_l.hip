// Column-pass instances for the long axes (256, 512 and 1024 points).
#include "passes_col.h"

namespace pat {

hipError_t launch_col_long(const ColSpec& spec, ColVariant v, int na, const Launch& L) {
  switch (na) {
    case 256: return launch_col_na<256>(spec, v, L);
    case 512: return launch_col_na<512>(spec, v, L);
    case 1024: return launch_col_na<1024>(spec, v, L);
  }
  return hipErrorInvalidValue;
}

hipError_t upload_twiddles_cols_long(const Tw* host) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host, sizeof(Tw) * TWN, 0, hipMemcpyHostToDevice);
}

}  // namespace pat
