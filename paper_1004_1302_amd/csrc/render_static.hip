// splotch_render_static: splotch_render for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  Its workspace is a file-scope device
// array of SPLOTCH_STATIC_SCRATCH_BYTES, one copy per GPU, held until the
// process ends; the caller passes only the particles, palette and image.
#include <map>
#include <mutex>

#include "../../include/splotch.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = SPLOTCH_STATIC_SCRATCH_BYTES;

// The render's workspace for this entry point.  In host code `scratch`
// names a host-side stand-in, never the device memory: host code uses only
// the per-device address that hipGetSymbolAddress returns.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, void *> g_addr;  // device -> address of that device's copy

// Address of the current device's copy, looked up once per device (with
// that device current).
splotch_status scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPLOTCH_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_addr.find(dev);
    if (it == g_addr.end()) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return SPLOTCH_E_DEVICE;
        it = g_addr.emplace(dev, p).first;
    }
    *out = it->second;
    return SPLOTCH_OK;
}

}  // namespace

extern "C" splotch_status splotch_render_static(const splotch_particles *particles,
                                                const splotch_camera *cam,
                                                const splotch_colourmap *cmap,
                                                const splotch_params *params,
                                                splotch_image *image) {
    if (!particles || !params) return SPLOTCH_E_INVALID_ARG;
    // stage timing creates HIP events: not offered here
    if (params->profile) return SPLOTCH_E_INVALID_ARG;
    // the smallest layout (one pair slot per pass) must fit; more pairs
    // than the scratch holds are rendered in several passes
    size_t need = 0;
    splotch_status st = splotch_workspace_size(particles->n, cam, params, 1, &need);
    if (st != SPLOTCH_OK) return st;
    if (need > kScratchBytes) return SPLOTCH_E_SCRATCH;
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != SPLOTCH_OK) return st;
    splotch_params q = *params;
    q.workspace = ws;
    q.workspace_bytes = kScratchBytes;
    return splotch_render(particles, cam, cmap, &q, image);
}
