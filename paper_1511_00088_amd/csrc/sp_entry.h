// Helpers shared by the C-ABI source files (sp_api.hip, sp_noalloc.hip): argument checks and the enqueue
// part of the gradient entry points, and the per-thread error message.
#pragma once

#include "../../include/sp_api.h"
#include "sp_launch.h"

namespace sp {

// Records msg as the calling thread's last error (sp_last_error) and returns code.
int set_error(int code, const char* msg);

// Validates an sp_geom (even extents >= 2, V/2 < 2^24, bc_t 0 or 1) and fills G; returns an sp_status.
int geom_check(const sp_geom* g, Geom* G);

// The tuned launch shape of the half operator for (G, link precision, recon, vector precision), or the default.
LaunchCfg tuned_launch(const Geom& G, int lp, int recon, int vp);

// Checks of sp_cg_force's arguments (geometry, null pointers, finite mass); fills G.
int force_check(const sp_geom* g, const sp_gauge* U, double mass, const double* x_e, const double* lambda_e,
                const double* gamma, Geom* G);

// Scratch bytes of the gradient's launches on G (what sp_force_workspace_bytes reports).
size_t force_scratch_bytes(const Geom& G);

// Enqueues the gradient's launches on s with their scratch at base (256-byte aligned, force_scratch_bytes(G)
// bytes); returns an sp_status.
int force_enqueue(const sp_geom* g, const Geom& G, const sp_gauge* U, double mass, const double* x_e,
                  const double* lambda_e, double* gamma, double* force, double* grad_mass, char* base, hipStream_t s);

}  // namespace sp
