// Serving entry points (continuous batching).  Placeholder until the
// persistent-kernel server lands: every call reports VDI_ERR_STATE.
#include <hip/hip_runtime.h>

#include "vdi_internal.h"

extern "C" {
int vdi_server_create(uint64_t, int32_t, int32_t, vdi_server_t *) { return VDI_ERR_STATE; }
int vdi_server_submit(vdi_server_t, vdi_t, const vdi_camera *, int32_t, int32_t, float, float, float *, uint64_t *)
{
    return VDI_ERR_STATE;
}
int vdi_server_poll(vdi_server_t, uint64_t, int *) { return VDI_ERR_STATE; }
int vdi_server_drain(vdi_server_t) { return VDI_ERR_STATE; }
int vdi_server_get_stats(vdi_server_t, vdi_server_stats *) { return VDI_ERR_STATE; }
int vdi_server_destroy(vdi_server_t) { return VDI_OK; }
}
