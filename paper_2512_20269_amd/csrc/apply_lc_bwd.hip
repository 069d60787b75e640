// Instantiations of the IFFD line pass: FFT lengths 128, backward passes.
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(128, PASS_BWD);

}  // namespace iffd
