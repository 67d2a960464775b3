#include "mf_resident.hpp"
namespace mf {
bool resident_supported(int, int) { return false; }
hipError_t launch_resident_sample(int, const ResidentArgs&, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace mf
