// Instantiations of the IFFD line pass: FFT lengths 64, 96, middle passes (forward, scaling, backward).
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(64, PASS_MID);
template IFFD_LINE_PASS_MODE(96, PASS_MID);

}  // namespace iffd
