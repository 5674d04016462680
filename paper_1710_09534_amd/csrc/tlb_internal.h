// tlb_internal.h -- structures shared by the host runtime and the gfx950
// kernels of the ternary wetting lattice Boltzmann library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tlb {

constexpr int kMaxMaterials = 15;
constexpr int kTileX = 64;        // interior columns per workgroup (one wave64 row)
constexpr int kThreads = 256;     // four wave64s per workgroup (auxiliary kernels)
constexpr int kReduceBlocks = 512;
constexpr int kScratchDoubles = kReduceBlocks * 4;   // static scratch of tlb_mass_noalloc
constexpr int kMaxDevices = 64;

enum Precision : int { P64 = 0, P32 = 1, P16 = 2 };

// Device views of the state.  Populations are stored SoA as 27 planes
// q = fam*9 + k (fam 0: f^1, 1: f^2, 2: g), each plane npad elements with
// row pitch `pitch`.  In P16 mode the rest planes q = 0 and q = 9 live in
// the float array `rest` (two planes), the other f^1, f^2 planes are FP16
// values multiplied by scale[fam] (paired per direction in 32-bit words) and
// the nine g planes are FP32.
struct PopBuf {
    void* planes;   // element type: double (P64), float (P32), _Float16 (P16)
    float* rest;    // P16 only
};

// Constants of one solve, precomputed on the host in FP64 and rounded to
// the arithmetic type of the kernel.
template <typename R>
struct Consts {
    R drho1, drho2, rho3;        // rho = rho3 + (rho1-rho3) c1 + (rho2-rho3) c2 (Eq. 14)
    R dnu1, dnu2, nu3;           // Eq. 15
    R itau1, itau2;              // 1/tau_i
    R fs1, fs2;                  // 1 - 1/(2 tau_i) (Eq. 11a)
    R eta1, eta2;                // Eq. 18a per component
    R am1, am2;                  // (rho_i - rho_3) M_i (Eq. 12)
    R lam1, lam2, lam3, lamT;    // Eqs. 7, 9
    R k12D, k34D, k4D;           // 12/D, 3D/4, 4/D
    R gx, gy;                    // gravity
    float scale[3], iscale[3];   // P16 storage scales of f^1, f^2 (g: 1)
    unsigned nee;                // bit m set: material m is a velocity boundary
                                 // (non-equilibrium extrapolation, Eqs. 51-53)
    // fields used only by optional kernel parts stay last, so that adding
    // them leaves the layout the plain step kernel loads unchanged
    R kB;                        // 8 lambda lambda_T / D (lambda c1^2 c2^2 c3^2 term of Eq. 5)
    R il1, il2, il3;             // 1 / lambda_i
};

// Per-material table (device memory, FP64): for material id m in 0..15 the
// five values cos(theta12), cos(theta13), cos(theta23), u_wall_x, u_wall_y at
// mtab[5*m .. 5*m+4]; id 0 (fluid) is all zero.  For a velocity boundary
// material the cosines are 0 and (u_wall_x, u_wall_y) is the boundary velocity.
constexpr int kMatStride = 5;

struct Grid {
    int nx, ny, pitch;
    long npad;                   // ny * pitch
    int tiles_x, tiles_y, tile_rows;
};

// Device descriptor of one lattice for the step kernel (R: arithmetic type,
// H: history storage type).  buf[cur] holds the current state at the step
// the launch's parity 0 refers to.  Of the two sets of history planes,
// hist[hcur ^ (bit 1 of the launch's parity)] holds the current history: the
// one-step kernel updates it in place, the two-step kernel writes the other
// set (another strip may still read the old one).
template <typename R, typename H>
struct LatDesc {
    Grid g;
    Consts<R> c;
    const uint8_t* mat;
    const double* mtab;
    PopBuf buf[2];
    H* hist[2];
    int tile_begin;   // prefix sum of the strip counts of the preceding lattices
    int cur;
    int hcur;
    int pair_rows;        // strip rows of the two-step kernel (0: not used)
    int pair_tile_begin;  // prefix sum of the preceding lattices' two-step strips
};
// A descriptor table stores descriptor i at byte offset i * kDescBytes.
constexpr size_t kDescBytes = 512;  // >= sizeof(LatDesc), a multiple of 256

// host-side launchers (tlb_kernels.hip)
// Step kernel over a device table of descriptors (LatDesc<double,double> for
// P64, LatDesc<float,float> otherwise); total_tiles = sum of strip counts;
// features: bit 0 some lattice of the table has velocity boundary nodes,
// bit 1 some lattice has a bulk energy with lambda > 0; parity bit 0 selects
// the population buffer, bit 1 the history set (see LatDesc).
hipError_t launch_step(int prec, unsigned features, const void* descs, int ndesc,
                       int total_tiles, int parity, hipStream_t s);
// Two steps per launch over a table of ndesc lattices (P32, any width;
// features as for launch_step): each descriptor's pair_rows (a multiple
// of 4) and pair_tile_begin give its strips, total_tiles their sum; the
// populations land in the buffer the first of two step_kernel launches would
// have written, the history in the set the launch's parity does not select.
hipError_t launch_step2(int prec, unsigned features, const void* descs, int ndesc,
                        int total_tiles, int parity, hipStream_t s);
// `consts` points to a host Consts<double> (P64) or Consts<float> (P32, P16);
// `mtab` to the device material table.
hipError_t launch_init(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                       const double* mtab, const double* in4, PopBuf dst, void* hist,
                       hipStream_t s);
// fields of the rows [ya, yb): out10[10][(yb - ya) * nx]
hipError_t launch_readout(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                          const double* mtab, PopBuf src, int ya, int yb, double* out10,
                          hipStream_t s);
// populations of the rows [ya, yb): out27[27][(yb - ya) * nx]
hipError_t launch_populations(int prec, const Grid& g, const void* consts,
                              const uint8_t* mat, PopBuf src, int ya, int yb, double* out27,
                              hipStream_t s);
// per-component mass and health of the history planes `hist` (double in P64,
// float otherwise): result[0..3] = sum c1, sum c2, sum c3 over fluid nodes and
// the count of nodes with a non-finite c1, c2, ux or uy; partials holds
// kReduceBlocks * 4 doubles
hipError_t launch_mass(int prec, const Grid& g, const uint8_t* mat, const void* hist,
                       double* partials, double* result, hipStream_t s);
// device address of the current GPU's copy of the static partial-sum array
// (kScratchDoubles doubles), resolved once per device
hipError_t mass_scratch(double** out);

}  // namespace tlb

struct tlb_ctx;
namespace tlb {
// queues the mass/health reduction of a context on stream s (which must be
// ordered after the context's last step) and the copy of its four results
// (sum c1, c2, c3, non-finite count) to pinned host memory host4; the
// serving loop uses it to check running requests behind their quantum
int health_enqueue(tlb_ctx* c, hipStream_t s, double* host4);

}  // namespace tlb
