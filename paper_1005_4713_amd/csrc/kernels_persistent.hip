// kernels_persistent.hip -- the persistent ("PERSISTENT") engine.
#include <string>

#include "spkmc_device.hpp"

namespace spkmc {

bool persistent_supported(const Geom &g, const spkmc_params &p, std::string &why) {
    (void)g;
    (void)p;
    why = "not built yet";
    return false;
}

hipError_t persistent_configure(const Geom &, const spkmc_params &, int &, int &, int &) { return hipErrorNotSupported; }

hipError_t launch_persistent(const Geom &, uint64_t, uint64_t, uint32_t, int, int, int, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace spkmc
