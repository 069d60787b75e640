// Instantiations of the IFFD line pass: FFT lengths 128, forward passes.
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(128, PASS_FWD);

}  // namespace iffd
