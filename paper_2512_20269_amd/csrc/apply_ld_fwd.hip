// Instantiations of the IFFD line pass: FFT lengths 192, forward passes.
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(192, PASS_FWD);

}  // namespace iffd
