/*
 * tlb3d.h -- C ABI of the three-dimensional version of the ternary wetting
 * lattice Boltzmann step on one AMD Instinct MI355X (gfx950).
 *
 * The paper (Liang, Xu, Chen, Chai & Shi, arXiv:1710.09534) states its model
 * on D2Q9 without loss of generality (Sec. II.A).  This library carries every
 * equation to the D3Q19 lattice (rest, 6 axis links, 12 edge diagonals;
 * weights 1/3, 1/18, 1/36; c_s^2 = 1/3), link by link: moments, wetting
 * ghosts across wall links (Eq. 42), chemical potentials (Eq. 8; Eq. 6 when
 * lambda > 0), symmetric ghosts (Eq. 43), forces and velocity (Eq. 13b),
 * interfacial force (Eq. 12), pressure (Eq. 13c with w_0 = 1/3), equilibria
 * and sources (Eqs. 2, 4, 11), BGK collision (Eq. 45), half-way bounce-back
 * with the moving-wall term (Eq. 44).
 *
 * Conventions are those of tlb.h, with z added: host fields are doubles
 * indexed (z*ny + y)*nx + x, z = 0 is the bottom plane; material 0 is fluid,
 * m >= 1 a wall of material mats[m-1] (kind TLB_WALL only; wall velocity
 * (wall_u[0], wall_u[1], 0)); in a non-periodic direction every node on the
 * two boundary faces must be a wall.  Status codes, error order and
 * ownership are those of tlb.h.  Storage precision: TLB_FP64 or TLB_FP32
 * (TLB_FP16DEV is TLB_EINVAL here).
 */
#ifndef TLB3D_H
#define TLB3D_H

#include <stddef.h>
#include <stdint.h>

#include "tlb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* field bits of tlb3_read_fields; fields are written in this bit order */
enum {
    TLB3_F_C1 = 1u << 0, TLB3_F_C2 = 1u << 1, TLB3_F_C3 = 1u << 2, TLB3_F_RHO = 1u << 3,
    TLB3_F_UX = 1u << 4, TLB3_F_UY = 1u << 5, TLB3_F_UZ = 1u << 6, TLB3_F_P = 1u << 7,
    TLB3_F_MU1 = 1u << 8, TLB3_F_MU2 = 1u << 9, TLB3_F_MU3 = 1u << 10,
    TLB3_F_ALL = (1u << 11) - 1
};

typedef struct tlb3_ctx tlb3_ctx;

/* Device workspace for an nx x ny x nz lattice (bytes); 0 for a dimension
 * < 3, nz > 65535, an unsupported precision, or a lattice beyond the size
 * limit of tlb3_create. */
size_t tlb3_workspace_bytes(int nx, int ny, int nz, tlb_precision p);

/* Create a context on a caller-owned device workspace (>= tlb3_workspace_bytes,
 * 256-byte aligned, alive until tlb3_destroy) and a HIP stream (NULL =
 * default).  fl: as in tlb_create (same validation); gravity = (fl->gravity[0],
 * fl->gravity[1], gravity_z).  Each family of 19 population planes must stay
 * below 2 GiB, counted with rows padded to a multiple of 64 nodes: at most
 * about 14.1 M nodes in FP64 (e.g. 192 x 240 x 300), 28.2 M in FP32; a larger
 * lattice, or nz > 65535, is TLB_EINVAL. */
tlb_status tlb3_create(int nx, int ny, int nz, tlb_precision p, const tlb_fluid* fl,
                       double gravity_z, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                       tlb3_ctx** out);

/* Wall geometry and wettability: material host uint8 [nz*ny*nx]; theta12 of
 * each material from Eq. 39 into theta12_out[n_mats] (nullable).  A material
 * kind other than TLB_WALL, or a fluid node on the face of a non-periodic
 * direction, is TLB_EINVAL; |cos theta12| > 1 is TLB_EPARAM. */
tlb_status tlb3_set_geometry(tlb3_ctx* ctx, int periodic_x, int periodic_y, int periodic_z,
                             const uint8_t* material, const tlb_material* mats, int n_mats,
                             double* theta12_out);

/* Initial order parameters and velocity (host [nz*ny*nx]; ux/uy/uz NULL = 0):
 * equilibrium populations with the chemical potentials of the initial field
 * and p = 0, history (c1, c2, u).  Synchronous. */
tlb_status tlb3_init_fields(tlb3_ctx* ctx, const double* c1, const double* c2,
                            const double* ux, const double* uy, const double* uz);

/* Advance nsteps steps asynchronously on the context's stream; a device
 * mass/NaN check runs every check_interval steps (default 100, 0 = never)
 * and a NaN/Inf order parameter makes a later call return TLB_EDIVERGED. */
tlb_status tlb3_step(tlb3_ctx* ctx, int64_t nsteps);
tlb_status tlb3_set_check_interval(tlb3_ctx* ctx, int64_t interval);

/* Macroscopic fields (TLB3_F_* bits, in bit order) into host_out
 * [popcount(mask) * nz*ny*nx]; walls read 0.  Synchronous. */
tlb_status tlb3_read_fields(tlb3_ctx* ctx, uint32_t field_mask, double* host_out);

/* Populations f(x, t) as doubles: f^1_0..18, f^2_0..18, g_0..18, each
 * [nz*ny*nx]; walls read 0.  Synchronous. */
tlb_status tlb3_read_populations(tlb3_ctx* ctx, double* host_out);

/* sum of c1, c2, c3 over fluid nodes (FP64, fixed order).  Synchronous;
 * TLB_EDIVERGED on NaN/Inf. */
tlb_status tlb3_mass(tlb3_ctx* ctx, double out[3]);

/* Device time per step (ms) of nsteps steps, by HIP events on the
 * context's stream (no health checks inside). */
tlb_status tlb3_time_steps(tlb3_ctx* ctx, int64_t nsteps, double* ms_per_step);

const char* tlb3_last_error(const tlb3_ctx* ctx);
void tlb3_destroy(tlb3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TLB3D_H */
