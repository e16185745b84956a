// Status strings, version and the per-thread HIP error slot of the C ABI.
#include "plic_host.hpp"

namespace plic {
namespace {
thread_local int g_last_hip_error = 0;
}
void set_last_hip_error(int e) { g_last_hip_error = e; }
}  // namespace plic

extern "C" {

const char* plic_status_string(int status) {
    switch (status) {
        case PLIC_OK: return "PLIC_OK: success";
        case PLIC_EINVAL: return "PLIC_EINVAL: invalid argument (null, misaligned or overlapping pointer, negative size or unknown enum)";
        case PLIC_EHIP: return "PLIC_EHIP: the HIP runtime rejected the launch";
        case PLIC_EWORKSPACE: return "PLIC_EWORKSPACE: the workspace is too small for this call";
        default: return "unknown PLIC status";
    }
}

const char* plic_version(void) { return "plic-mi355x 0.1.0 (gfx950)"; }

int plic_last_hip_error(void) { return plic::g_last_hip_error; }

}  // extern "C"
