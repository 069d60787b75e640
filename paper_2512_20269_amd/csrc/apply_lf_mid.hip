// Instantiations of the IFFD line pass: FFT length 384, middle passes (forward, scaling, backward).
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(384, PASS_MID);

}  // namespace iffd
