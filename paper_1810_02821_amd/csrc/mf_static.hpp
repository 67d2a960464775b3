// Static device scratch of mf_sample_noalloc (defined in mf_static.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mf {

// Size of the static scratch array, per GPU; held until the process ends.
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;

// Record the scratch array's address on `device`, which must be the current
// device (once per device; later calls return at once).
hipError_t static_scratch_setup(int device);
// The scratch address on `device`, or nullptr before static_scratch_setup.
void* static_scratch(int device);

}  // namespace mf
