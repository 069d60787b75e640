// Instantiations of the IFFD line pass: FFT lengths 256, middle passes (forward, scaling, backward).
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(256, PASS_MID);

}  // namespace iffd
