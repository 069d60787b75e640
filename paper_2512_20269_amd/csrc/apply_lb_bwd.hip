// Instantiations of the IFFD line pass: FFT lengths 64, 96, backward passes.
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(64, PASS_BWD);
template IFFD_LINE_PASS_MODE(96, PASS_BWD);

}  // namespace iffd
