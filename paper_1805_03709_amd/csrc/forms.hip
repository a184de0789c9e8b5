// The boundary's generic forms, composed from the specific calls: live keys of a map, the
// sticky error of either kind of handle, and the MC extraction of every allocated block.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "host.hpp"
#include "vbh.h"

using namespace vbh;

extern "C" {

int vbh_size(vbh_map *m, int64_t *h_size, void *stream) {
    if (!h_size) return VBH_EINVAL;
    int64_t tomb = 0;
    return vbh_map_size(m, h_size, &tomb, stream);
}

int vbh_status(void *handle, void *stream) {
    if (!handle) return VBH_EINVAL;
    const uint32_t tag = *static_cast<const uint32_t *>(handle);
    if (tag == kTagMap) return vbh_map_status(static_cast<vbh_map *>(handle), stream);
    if (tag == kTagScene) return vbh_scene_status(static_cast<vbh_scene *>(handle), stream);
    return VBH_EINVAL;
}

int vbh_extract_mc_all(vbh_scene *s, int32_t *d_keys_out, int64_t cap, uint8_t *d_mc, uint8_t *d_rgb,
                       int64_t *h_count, void *stream) {
    if (!s || !h_count || cap < 0 || (cap > 0 && (!d_keys_out || !d_mc))) return VBH_EINVAL;
    const int rc = vbh_scene_export_blocks(s, d_keys_out, cap, h_count, stream);
    if (rc != VBH_OK) return rc;
    return vbh_extract_mc_indices(s, d_keys_out, std::min(cap, *h_count), d_mc, d_rgb, stream);
}

}  // extern "C"
