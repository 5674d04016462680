// tlb3d_internal.h -- structures shared by the host runtime and the gfx950
// kernels of the three-dimensional (D3Q19) version of the ternary wetting
// lattice Boltzmann step.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tlb3 {

constexpr int kQ = 19;             // D3Q19
constexpr int kMaxMaterials = 15;
constexpr int kMatStride = 5;      // cos12, cos13, cos23, u_wall_x, u_wall_y (FP64)
constexpr int kBlockX = 64;        // a block covers 64 x-columns ...
constexpr int kBlockY = 4;         // ... of 4 rows of one z-plane
constexpr int kReduceBlocks = 512;

// Lattice geometry: node (x, y, z) at ((z * ny) + y) * pitch + x of every
// plane; pitch is nx rounded up to 64; npad = pitch * ny * nz.
struct Grid3 {
    int nx, ny, nz, pitch;
    long long npad;
};

// Constants of one solve in the arithmetic type R.
template <typename R>
struct Consts3 {
    R drho1, drho2, rho3;        // Eq. 14
    R dnu1, dnu2, nu3;           // Eq. 15
    R itau1, itau2, fs1, fs2;    // 1/tau_i, 1 - 1/(2 tau_i)
    R eta1, eta2;                // Eq. 18a per component
    R am1, am2;                  // (rho_i - rho_3) M_i (Eq. 12)
    R lam1, lam2, lam3, lamT;    // Eqs. 7, 9
    R k12D, k34D, k4D;           // 12/D, 3D/4, 4/D
    R gx, gy, gz;                // gravity
    R kB, il1, il2, il3;         // lambda > 0 part of Eq. 6: 8 lambda lambda_T / D, 1/lambda_i
};

// Device buffers of one lattice.  pop[b]: 57 planes (f^1_0..18, f^2_0..18,
// g_0..18); a plane slot P_k[y] holds the post-collision f'_k(y), so node x
// pulls P_k[x - e_k].  hist: c1, c2, ux, uy, uz of the previous step.  cf:
// c1, c2; muf: mu1, mu2, mu3 of the current step.
template <typename R>
struct Bufs3 {
    R* pop[2];
    R* hist;
    R* cf;
    R* muf;
    const uint8_t* mat;
    const double* mtab;
};

hipError_t launch3_step(int prec, const Grid3& g, const void* consts, const void* bufs, int cur,
                        hipStream_t s);
// order parameters into cf from the populations of buffer cur, then mu
hipError_t launch3_c_mu(int prec, const Grid3& g, const void* consts, const void* bufs, int cur,
                        hipStream_t s);
// init: cf from in5 (c1, c2 as doubles, n = nx*ny*nz each), then mu, then
// equilibrium populations into buffer 0 and history from in5 (ux, uy, uz)
hipError_t launch3_init(int prec, const Grid3& g, const void* consts, const void* bufs,
                        const double* in5, hipStream_t s);
// fields c1 c2 c3 rho ux uy uz p mu1 mu2 mu3 of buffer cur on the planes
// [za, zb) (11 x nx*ny*(zb-za) doubles); launch3_c_mu must have run on cur
hipError_t launch3_readout(int prec, const Grid3& g, const void* consts, const void* bufs,
                           int cur, int za, int zb, double* out11, hipStream_t s);
// populations of family fam (f^1, f^2, g) of buffer cur on the planes
// [za, zb): 19 x nx*ny*(zb-za) doubles
hipError_t launch3_populations(int prec, const Grid3& g, const void* bufs, int cur, int fam,
                               int za, int zb, double* out19, hipStream_t s);
hipError_t launch3_mass(int prec, const Grid3& g, const void* bufs, int cur, double* partials,
                        double* result, hipStream_t s);

}  // namespace tlb3
