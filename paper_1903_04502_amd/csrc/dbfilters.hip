// Daubechies filters for the SARA dictionary (Section "Analysis and
// Synthesis"): the host spectral factorisation in host/daubechies.hpp.
#include "host/daubechies.hpp"
#include "psi.hpp"

namespace pr {

bool daubechies_filter(int N, double* h) { return host::daubechies_filter(N, h); }

}  // namespace pr
