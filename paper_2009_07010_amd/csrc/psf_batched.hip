// Batched persistent path (placeholder until the persistent kernel lands).
#include "psf_host.hpp"

namespace psf {
size_t batched_workspace(const psf_obs*, int, const psf_src*, int) { return 0; }
}  // namespace psf

using namespace psf;
extern "C" {
int psf_patch_batched(const psf_obs*, int32_t, const psf_src*, const psf_src*, int, const char*, float*, void*,
                      size_t, void*) {
  return fail(PSF_EUNSUPPORTED, "psf_patch_batched not built yet");
}
int psf_autotune(const psf_obs*, int32_t, const psf_src*, int, void*, size_t, char*, size_t, void*) {
  return fail(PSF_EUNSUPPORTED, "psf_autotune not built yet");
}
}
