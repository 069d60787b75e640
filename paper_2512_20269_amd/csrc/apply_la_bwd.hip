// Instantiations of the IFFD line pass: FFT lengths 16, 24, 32, 48, backward passes.
#include "apply_impl.h"

namespace iffd {

template IFFD_LINE_PASS_MODE(16, PASS_BWD);
template IFFD_LINE_PASS_MODE(24, PASS_BWD);
template IFFD_LINE_PASS_MODE(32, PASS_BWD);
template IFFD_LINE_PASS_MODE(48, PASS_BWD);

}  // namespace iffd
