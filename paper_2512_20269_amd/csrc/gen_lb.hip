// Instantiations of the general-plan line passes: FFT lengths 64, 96.
#include "gen_impl.h"

namespace iffd {

template IFFD_GEN_PASS_LEN(64);
template IFFD_GEN_PASS_LEN(96);

}  // namespace iffd
