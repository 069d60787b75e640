// Instantiations of the general-plan line passes: FFT lengths 192.
#include "gen_impl.h"

namespace iffd {

template IFFD_GEN_PASS_LEN(192);

}  // namespace iffd
