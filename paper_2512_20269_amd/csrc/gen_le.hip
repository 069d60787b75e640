// Instantiations of the general-plan line passes: FFT lengths 256.
#include "gen_impl.h"

namespace iffd {

template IFFD_GEN_PASS_LEN(256);

}  // namespace iffd
