// Instantiations of the general-plan line passes: FFT lengths 16, 24, 32, 48.
#include "gen_impl.h"

namespace iffd {

template IFFD_GEN_PASS_LEN(16);
template IFFD_GEN_PASS_LEN(24);
template IFFD_GEN_PASS_LEN(32);
template IFFD_GEN_PASS_LEN(48);

}  // namespace iffd
