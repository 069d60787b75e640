// Instantiations of the IFFD line pass: FFT length 384, forward passes.
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(384, PASS_FWD);

}  // namespace iffd
