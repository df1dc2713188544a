// Serving loop (continuous batching with HBM-footprint admission).
#include "bc_internal.h"

extern "C" {
bc_status bc_serve_create(size_t, int32_t, bc_server*) { return BC_E_STATE; }
bc_status bc_serve_submit(bc_server, bc_graph, const uint32_t*, int32_t, double*, uint64_t*) { return BC_E_STATE; }
bc_status bc_serve_poll(bc_server, uint64_t, bc_info*) { return BC_E_STATE; }
bc_status bc_serve_destroy(bc_server) { return BC_E_STATE; }
}
