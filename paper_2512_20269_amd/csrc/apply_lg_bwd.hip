// Instantiations of the IFFD line pass: FFT length 512, backward passes.
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(512, PASS_BWD);

}  // namespace iffd
