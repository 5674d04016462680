// tlb_kernels.hip -- gfx950 kernels of the ternary wetting lattice Boltzmann
// step (Liang et al., arXiv:1710.09534, Sec. II).
//
// Data layout (HBM): 27 SoA population planes per lattice, row pitch a
// multiple of 64 nodes, two lattices (ping-pong).  A plane slot P_k[y] holds
// the post-collision population f'_k(y) of the previous step, so the
// population entering node x along e_k is P_k[x - e_k] (pull streaming).
// Half-way bounce-back (Eq. 44) is folded into the store: a fluid node whose
// neighbour x + e_k is solid also writes f'_k(x) (plus the moving-wall term)
// into slot P_{opp(k)} of that solid node, which only x ever pulls from, so
// the pull needs no per-link branch.
//
// One step is one kernel (step_kernel below).  A workgroup marches up a
// strip of 64 columns, and per group of four rows
//   A. pulls f^1, f^2 and forms c1, c2 into an LDS ring (Eqs. 3, 13a),
//   B. forms the chemical potentials with the wetting ghosts of Eq. 42
//      across solid links (Eqs. 8, 20b),
//   C. per node: gradients with the symmetric ghost rule (Eq. 43),
//      surface-tension force, velocity, interfacial force, pressure,
//      Euler time derivative, equilibria, sources and BGK collision
//      (Eqs. 2, 4, 11-15, 18b, 19, 45), and the coalesced stores.
// Workgroup ids are remapped so that each of the eight XCDs walks one
// contiguous band of strips: side-halo re-reads then hit that XCD's L2.
// The init and readout kernels use a plain 64 x 8 tile with a 2-node halo.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tlb_internal.h"

// Partial sums of the mass reduction for tlb_mass_noalloc, the entry point for
// callers that cannot allocate: a fixed array in device memory (16 KiB), one
// copy per GPU, kept until the process ends and shared by every such call on
// that GPU.  In host code the array's name is only a host-side stand-in:
// tlb::mass_scratch() gives the device address of the current GPU's copy.
static __device__ __align__(256) double scratch[tlb::kScratchDoubles];

namespace tlb {
namespace {

// D2Q9 (Eq. 10)
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <typename R>
__device__ __forceinline__ constexpr R wgt(int k) {
    return k == 0 ? R(4) / R(9) : (k < 5 ? R(1) / R(9) : R(1) / R(36));
}

template <int P> struct Tr;
template <> struct Tr<P64> { using R = double; using S = double; using H = double; };
template <> struct Tr<P32> { using R = float; using S = float; using H = float; };
template <> struct Tr<P16> { using R = float; using S = _Float16; using H = float; };

// FP16-dev population buffer: f^1_k and f^2_k (k = 1..8) share one 32-bit
// word (f^1 in the low half) in 8 pair planes, followed by the 9 FP32 g
// planes; f^1_0 and f^2_0 live in the FP32 rest planes.  Halfword index of
// an order-parameter population q = 9 f + k (f: f^1, f^2; k >= 1) at node i:
template <int P>
__device__ __forceinline__ long half_index(int q, long npad, long i) {
    const int k = q % 9;
    return 2 * ((k - 1) * npad + i) + (q / 9);
}

template <int P>
__device__ __forceinline__ typename Tr<P>::R ld(const PopBuf& b, const Consts<typename Tr<P>::R>& c,
                                                int q, long npad, long i) {
    if constexpr (P == P16) {
        if (q == 0 || q == 9) return b.rest[(q / 9) * npad + i];
        if (q >= 18) return static_cast<const float*>(b.planes)[(8 + q - 18) * npad + i];
        return float(static_cast<const _Float16*>(b.planes)[half_index<P>(q, npad, i)]) *
               c.iscale[q / 9];
    } else {
        return static_cast<const typename Tr<P>::S*>(b.planes)[q * npad + i];
    }
}

template <int P>
__device__ __forceinline__ void st(const PopBuf& b, const Consts<typename Tr<P>::R>& c, int q,
                                   long npad, long i, typename Tr<P>::R v) {
    if constexpr (P == P16) {
        if (q == 0 || q == 9) {
            b.rest[(q / 9) * npad + i] = v;
        } else if (q >= 18) {
            static_cast<float*>(b.planes)[(8 + q - 18) * npad + i] = v;
        } else {
            static_cast<_Float16*>(b.planes)[half_index<P>(q, npad, i)] =
                _Float16(v * c.scale[q / 9]);
        }
    } else {
        static_cast<typename Tr<P>::S*>(b.planes)[q * npad + i] = v;
    }
}

__device__ __forceinline__ int wrapc(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Node neighbourhood in the periodic index space: columns x-1, x, x+1 and
// row offsets of y-1, y, y+1.
struct Nb {
    int xm, x0, xp;
    long rm, r0, rp;
    __device__ __forceinline__ long at(int dx, int dy) const {
        long r = dy < 0 ? rm : (dy > 0 ? rp : r0);
        int x = dx < 0 ? xm : (dx > 0 ? xp : x0);
        return r + x;
    }
    // slot pulled by direction k: x - e_k
    __device__ __forceinline__ long up(int k) const { return at(-EX[k], -EY[k]); }
    // neighbour along e_k
    __device__ __forceinline__ long dn(int k) const { return at(EX[k], EY[k]); }
};

__device__ __forceinline__ Nb make_nb(const Grid& g, int x, int y) {
    Nb n;
    n.x0 = x;
    n.xm = x == 0 ? g.nx - 1 : x - 1;
    n.xp = x == g.nx - 1 ? 0 : x + 1;
    n.r0 = long(y) * g.pitch;
    n.rm = long(y == 0 ? g.ny - 1 : y - 1) * g.pitch;
    n.rp = long(y == g.ny - 1 ? 0 : y + 1) * g.pitch;
    return n;
}

template <int P, int TY>
struct Smem {
    using R = typename Tr<P>::R;
    static constexpr int CW = kTileX + 4, CH = TY + 4;   // c region: tile + 2-node halo
    static constexpr int MW = kTileX + 2, MH = TY + 2;   // mu region: tile + 1-node halo
    R c1[CH * CW];
    R c2[CH * CW];
    R mu1[MH * MW];
    R mu2[MH * MW];
    R mu3[MH * MW];
    R mt[kMatStride * (kMaxMaterials + 1)];
    uint8_t m[CH * CW];
};

// XCD-aware tile order: workgroup L runs on XCD L % 8; give XCD j the
// contiguous band of tiles [j*per, (j+1)*per).
__device__ __forceinline__ int tile_of(int L, int ntiles) {
    if (ntiles % 8) return L;
    int per = ntiles / 8;
    return (L % 8) * per + L / 8;
}

template <int P, int TY>
__device__ __forceinline__ void load_mtab(Smem<P, TY>& sm, const double* mtab) {
    for (int i = threadIdx.x; i < kMatStride * (kMaxMaterials + 1); i += kThreads)
        sm.mt[i] = typename Tr<P>::R(mtab[i]);
}

// Phase A: material ids and order parameters on the c region.  FROM_POPS
// pulls the populations (Eq. 13a); otherwise c comes from host input.
template <int P, int TY, bool FROM_POPS>
__device__ __forceinline__ void phase_a(Smem<P, TY>& sm, const Grid& g,
                                        const Consts<typename Tr<P>::R>& c, const uint8_t* mat,
                                        const PopBuf& src, const double* in4, int x0, int y0) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    for (int i = threadIdx.x; i < SM::CH * SM::CW; i += kThreads) {
        int ly = i / SM::CW;
        int lx = i - ly * SM::CW;
        int gx = wrapc(x0 - 2 + lx, g.nx);
        int gy = wrapc(y0 - 2 + ly, g.ny);
        long idx = long(gy) * g.pitch + gx;
        uint8_t m = mat[idx];
        sm.m[i] = m;
        R a = R(0), b = R(0);
        if (m == 0) {
            if constexpr (FROM_POPS) {
                Nb nb = make_nb(g, gx, gy);
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    long j = nb.up(k);
                    a += ld<P>(src, c, k, g.npad, j);
                    b += ld<P>(src, c, 9 + k, g.npad, j);
                }
            } else {
                long hi = long(gy) * g.nx + gx;
                long n = long(g.nx) * g.ny;
                a = R(in4[hi]);
                b = R(in4[n + hi]);
            }
        }
        sm.c1[i] = a;
        sm.c2[i] = b;
    }
}

// 1/x: FP32 arithmetic uses the hardware reciprocal (1 ulp), FP64 divides
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Macroscopic state of one interior node (phase C front half).
template <typename R>
struct NodeMacro {
    R c1, c2, rho, itg, mu1, mu2, ux, uy, p, grx, gry, fx, fy, fax, fay;
    R am;   // sum_i (rho_i - rho_3) M_i lap mu_i, so that F_a = u am (Eq. 12)
};

// Neighbour mask of a node (step kernel): bit k-1 for a wall neighbour along
// e_k, bit 8 when the node itself is not fluid, bit 15+k for a velocity
// boundary neighbour along e_k.
constexpr unsigned kWallBits = 0xFFu;
constexpr unsigned kSelfBit = 0x100u;
constexpr unsigned kVelShift = 15u;
constexpr unsigned kVelBits = 0xFFu << 16;

// Optional parts of the step, selected per launch at compile time so that a
// lattice that does not use them runs code without them.
constexpr unsigned kFeatVel = 1u;   // velocity boundary nodes (Eqs. 51-53)
constexpr unsigned kFeatLam = 2u;   // bulk energy with lambda > 0 (Eqs. 5-6)

// LDS neighbourhood of one node: row pointers for y-1, y, y+1 (index 0..2),
// each already offset to the node's column.
template <typename R>
struct Stencil {
    const R* c1[3];
    const R* c2[3];
    const uint8_t* m[3];
    const R* mu1[3];
    const R* mu2[3];
    R mu3;
};

// Gradients (Eq. 20a, symmetric ghosts of Eq. 43), forces, velocity
// (Eq. 13b), interfacial force (Eq. 12) and pressure (Eq. 13c) from the
// pulled g and the LDS fields.  A velocity boundary neighbour x + e_k shows
// the value of the fluid node inside it, x + (e_kx, 0) (chi(x_u) = chi(x_f),
// Eq. 53).  When MASK is true the neighbour mask (kWallBits, kVelBits)
// replaces the LDS material bytes; VEL false compiles velocity boundaries out.
template <typename R, bool MASK = false, bool VEL = true>
__device__ __forceinline__ NodeMacro<R> node_macro(const Stencil<R>& s, const Consts<R>& c,
                                                   const R* gg, unsigned mask = 0u) {
    NodeMacro<R> o;
    const R c1 = s.c1[1][0], c2 = s.c2[1][0];
    const R mu1 = s.mu1[1][0], mu2 = s.mu2[1][0], mu3 = s.mu3;
    R g1x = R(0), g1y = R(0), g2x = R(0), g2y = R(0), lm1 = R(0), lm2 = R(0);
    const bool any = MASK ? (mask & (VEL ? kWallBits | kVelBits : kWallBits)) != 0u : true;
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        const int r = EY[k] + 1;
        bool solid, vel;
        if constexpr (MASK) {
            solid = any && ((mask >> (k - 1)) & 1u) != 0u;
            vel = VEL && any && ((mask >> (kVelShift + k)) & 1u) != 0u;
        } else {
            const unsigned mn = s.m[r][EX[k]];
            vel = ((c.nee >> mn) & 1u) != 0u;
            solid = mn != 0u && !vel;
        }
        // value across the link: own value (wall), the same-row neighbour
        // (velocity boundary) or the neighbour itself; every row index is a
        // compile-time constant
        const R v1 = solid ? c1 : (vel ? s.c1[1][EX[k]] : s.c1[r][EX[k]]);
        const R v2 = solid ? c2 : (vel ? s.c2[1][EX[k]] : s.c2[r][EX[k]]);
        const R w1 = solid ? mu1 : (vel ? s.mu1[1][EX[k]] : s.mu1[r][EX[k]]);
        const R w2 = solid ? mu2 : (vel ? s.mu2[1][EX[k]] : s.mu2[r][EX[k]]);
        if (EX[k]) {
            g1x += wgt<R>(k) * R(EX[k]) * v1;
            g2x += wgt<R>(k) * R(EX[k]) * v2;
        }
        if (EY[k]) {
            g1y += wgt<R>(k) * R(EY[k]) * v1;
            g2y += wgt<R>(k) * R(EY[k]) * v2;
        }
        lm1 += wgt<R>(k) * (w1 - mu1);
        lm2 += wgt<R>(k) * (w2 - mu2);
    }
    g1x *= R(3); g1y *= R(3); g2x *= R(3); g2y *= R(3);   // 1 / c_s^2
    lm1 *= R(6); lm2 *= R(6);
    const R g3x = -(g1x + g2x), g3y = -(g1y + g2y);        // c3 = 1 - c1 - c2
    const R rho = c.rho3 + c.drho1 * c1 + c.drho2 * c2;    // Eq. 14
    const R nu = c.nu3 + c.dnu1 * c1 + c.dnu2 * c2;        // Eq. 15
    const R taug = R(3) * nu + R(0.5);                     // Eq. 18b
    const R grx = c.drho1 * g1x + c.drho2 * g2x;           // grad rho
    const R gry = c.drho1 * g1y + c.drho2 * g2y;
    const R fsx = mu1 * g1x + mu2 * g2x + mu3 * g3x;       // F_s
    const R fsy = mu1 * g1y + mu2 * g2y + mu3 * g3y;
    const R fx = fsx + rho * c.gx;
    const R fy = fsy + rho * c.gy;
    R mx = R(0), my = R(0), sum = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (EX[k]) mx += R(EX[k]) * gg[k];
        if (EY[k]) my += R(EY[k]) * gg[k];
        if (k) sum += gg[k];
    }
    const R irho = recip(rho);
    const R ux = (mx + R(0.5) * fx) * irho;
    const R uy = (my + R(0.5) * fy) * irho;
    const R a = c.am1 * lm1 + c.am2 * lm2;
    const R uu = ux * ux + uy * uy;
    // c_s^2/(1-w0) = 3/5; s_0(u) = -w0 u.u/(2 c_s^2) = -(2/3) u.u
    const R p = R(0.6) * (sum + R(0.5) * (ux * grx + uy * gry) - rho * (R(2) / R(3)) * uu);
    o.c1 = c1; o.c2 = c2; o.rho = rho; o.itg = recip(taug);
    o.mu1 = mu1; o.mu2 = mu2; o.ux = ux; o.uy = uy; o.p = p;
    o.grx = grx; o.gry = gry; o.fx = fx; o.fy = fy; o.fax = ux * a; o.fay = uy * a;
    o.am = a;
    return o;
}

template <int P, int TY>
__device__ __forceinline__ Stencil<typename Tr<P>::R> tile_stencil(const Smem<P, TY>& sm, int ci,
                                                                   int mi) {
    using SM = Smem<P, TY>;
    Stencil<typename Tr<P>::R> s;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        s.c1[r] = &sm.c1[ci + (r - 1) * SM::CW];
        s.c2[r] = &sm.c2[ci + (r - 1) * SM::CW];
        s.m[r] = &sm.m[ci + (r - 1) * SM::CW];
        s.mu1[r] = &sm.mu1[mi + (r - 1) * SM::MW];
        s.mu2[r] = &sm.mu2[mi + (r - 1) * SM::MW];
    }
    s.mu3 = sm.mu3[mi];
    return s;
}

// The part of Eq. 6 that comes from the lambda c1^2 c2^2 c3^2 term of the bulk
// energy (Eq. 5): with dP/dc_i = 2 lambda c_i c_j^2 c_k^2,
//   (4 lambda_T / D) sum_{j != i} (dP/dc_i - dP/dc_j) / lambda_j
//     = kB c1 c2 c3 sum_{j != i} c_k (c_j - c_i) / lambda_j,  kB = 8 lambda lambda_T / D.
// A uniform branch: lattices with lambda = 0 (Eq. 8) skip it.
template <typename R, bool LAM = true>
__device__ __forceinline__ void lambda_term(const Consts<R>& c, R c1, R c2, R& mu1, R& mu2,
                                            R& mu3) {
    if (LAM && c.kB != R(0)) {
        const R c3 = R(1) - c1 - c2;
        const R t = c.kB * c1 * c2 * c3;
        mu1 += t * (c3 * (c2 - c1) * c.il2 + c2 * (c3 - c1) * c.il3);
        mu2 += t * (c3 * (c1 - c2) * c.il1 + c1 * (c3 - c2) * c.il3);
        mu3 += t * (c2 * (c1 - c3) * c.il1 + c1 * (c2 - c3) * c.il2);
    }
}

// Chemical potentials of Eq. 8 at one fluid node from the c values of its
// 3x3 neighbourhood (row pointers as in Stencil), with the wetting ghosts of
// Eq. 42 across links into walls and, across a link into a velocity boundary
// node, the value of the fluid node inside it (Eq. 53).
template <typename R, bool VEL = true, bool LAM = true>
__device__ __forceinline__ void chem_pot(const R* const* c1r, const R* const* c2r,
                                         const uint8_t* const* mr, const R* mt,
                                         const Consts<R>& c, R& mu1, R& mu2, R& mu3) {
    const R c1 = c1r[1][0], c2 = c2r[1][0];
    const R c3 = R(1) - c1 - c2;
    R l1 = R(0), l2 = R(0), l3 = R(0);
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        const int r = EY[k] + 1;
        const int mn = mr[r][EX[k]];
        R n1, n2, n3;
        if (VEL && ((c.nee >> mn) & 1u)) {
            n1 = c1r[1][EX[k]];
            n2 = c2r[1][EX[k]];
            n3 = R(1) - n1 - n2;
        } else if (mn) {
            const R* t = &mt[kMatStride * mn];
            const R h1 = t[1] * c1 * c3 + t[0] * c1 * c2;
            const R h2 = -t[0] * c1 * c2 + t[2] * c2 * c3;
            const R h3 = -t[2] * c2 * c3 - t[1] * c1 * c3;
            n1 = c1 + c.k4D * h1;
            n2 = c2 + c.k4D * h2;
            n3 = c3 + c.k4D * h3;
        } else {
            n1 = c1r[r][EX[k]];
            n2 = c2r[r][EX[k]];
            n3 = R(1) - n1 - n2;
        }
        l1 += wgt<R>(k) * (n1 - c1);
        l2 += wgt<R>(k) * (n2 - c2);
        l3 += wgt<R>(k) * (n3 - c3);
    }
    l1 *= R(6);  // 2 / c_s^2
    l2 *= R(6);
    l3 *= R(6);
    const R tri = R(2) * c.lamT * c1 * c2 * (R(1) - c1 - c2);
    mu1 = c.k12D * (c.lam1 * c1 * (R(1) - c1) * (R(1) - R(2) * c1) - tri) - c.k34D * c.lam1 * l1;
    mu2 = c.k12D * (c.lam2 * c2 * (R(1) - c2) * (R(1) - R(2) * c2) - tri) - c.k34D * c.lam2 * l2;
    mu3 = c.k12D * (c.lam3 * c3 * (R(1) - c3) * (R(1) - R(2) * c3) - tri) - c.k34D * c.lam3 * l3;
    lambda_term<R, LAM>(c, c1, c2, mu1, mu2, mu3);
}

// Phase B of the tile kernels: chemical potentials on the mu region.
template <int P, int TY>
__device__ __forceinline__ void phase_b(Smem<P, TY>& sm, const Consts<typename Tr<P>::R>& c) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    for (int i = threadIdx.x; i < SM::MH * SM::MW; i += kThreads) {
        const int my = i / SM::MW;
        const int mx = i - my * SM::MW;
        const int ci = (my + 1) * SM::CW + mx + 1;
        R mu1 = R(0), mu2 = R(0), mu3 = R(0);
        if (sm.m[ci] == 0) {
            const R* c1r[3] = {&sm.c1[ci - SM::CW], &sm.c1[ci], &sm.c1[ci + SM::CW]};
            const R* c2r[3] = {&sm.c2[ci - SM::CW], &sm.c2[ci], &sm.c2[ci + SM::CW]};
            const uint8_t* mr[3] = {&sm.m[ci - SM::CW], &sm.m[ci], &sm.m[ci + SM::CW]};
            chem_pot<R>(c1r, c2r, mr, sm.mt, c, mu1, mu2, mu3);
        }
        sm.mu1[i] = mu1;
        sm.mu2[i] = mu2;
        sm.mu3[i] = mu3;
    }
}

// ------------------------------------------------------------------- step
// The step kernel marches a workgroup up a strip of 64 columns and H rows,
// four rows per iteration.  Waves 0..3 (the row waves) own the strip's 64
// columns, one lane per column, so every row of every plane is read and
// written as whole, aligned 64-node segments; wave 4 (the halo wave) forms c
// on the two columns either side of the strip.  c (rows y-2..y+5) and mu
// (rows y-1..y+4) live in LDS rings, so every population is pulled once per
// strip apart from the side halo and 4 rows per strip.
//   phase A: row wave w forms c1, c2 of row Y+2+w from its prefetched
//            pulls and issues the g / history loads of its phase-C row; the
//            halo wave does the same for the 16 halo nodes of rows Y+2..Y+5
//            and issues their next pulls.  The loads complete while the
//            workgroup runs phase B.
//   phase B: mu on rows Y+1..Y+4, and each node's solid-neighbour mask.
//   phase C: row wave w updates row Y + ((w+2) & 3): waves 0, 1 the row they
//            pulled in this iteration (still in registers), waves 2, 3 the
//            row they pulled in the previous one (parked in a per-wave,
//            double-buffered LDS stash).  Before it collides, a row wave
//            issues the pulls of row Y+6+w for the next iteration.
// The row waves and the halo wave run separate loops with the same barrier
// sequence, so the compiler's wait counts for each follow its own stores.
// Memory is addressed through buffer resources: one 32-bit lane offset per
// lattice direction serves all 27 planes, the plane offset rides in an SGPR.
// Every row-wave lane executes the same loads and the 31 main stores; a lane
// without a fluid output node stores at an offset beyond the buffer's record
// count, which the hardware discards, so no lane needs a branch around the
// stores and the wait counts never cover the previous row's stores.  (The
// host keeps every family buffer below 2 GiB, so that offset plus any plane
// offset stays outside the record count.)
constexpr int kStepThreads = 5 * kTileX;  // four row waves and the halo wave
constexpr unsigned kDiscard = 0x80000000u;  // byte offset of a discarded store
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, gfx9 family

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), kRsrcWord3);
}

template <int P>
struct LatView {
    rsrc_t fam[3];      // f^1, f^2, g: plane k of a family at byte offset k * pstride.  P16:
                        // fam[0], fam[1] hold the (f^1_k, f^2_k) pair planes k = 1..4 and
                        // 5..8 at offset ((k - 1) & 3) * ppstride, fam[2] the FP32 g planes
    rsrc_t rest;        // P16: FP32 rest planes f^1_0 (offset 0), f^2_0 (offset rstride)
    unsigned pstride;   // bytes per plane (P16: per FP32 g plane)
    unsigned ppstride;  // P16 pair-plane bytes
    unsigned rstride;   // P16 rest-plane bytes
};

template <int P>
__device__ __forceinline__ LatView<P> lat_view(const PopBuf& b, long npad) {
    using S = typename Tr<P>::S;
    LatView<P> v;
    const unsigned ps = unsigned(npad * long(P == P16 ? 4 : sizeof(S)));
    const char* base = static_cast<const char*>(b.planes);
    if constexpr (P == P16) {
        const unsigned pp = unsigned(npad * 4);
        v.fam[0] = make_rsrc(base, 4u * pp);
        v.fam[1] = make_rsrc(base + long(4) * pp, 4u * pp);
        v.fam[2] = make_rsrc(base + long(8) * pp, 9u * ps);
        v.ppstride = pp;
    } else {
#pragma unroll
        for (int f = 0; f < 3; ++f) v.fam[f] = make_rsrc(base + long(f) * 9 * ps, 9u * ps);
        v.ppstride = 0;
    }
    v.pstride = ps;
    v.rstride = unsigned(npad * 4);
    v.rest = make_rsrc(P == P16 ? static_cast<const void*>(b.rest) : static_cast<const void*>(base),
                       P == P16 ? 2u * v.rstride : ps);
    return v;
}

// Cache policy (the buffer instructions' policy operand: bit 1 nt, bit 4
// sc1).  Every population is written once per step and read once in the
// next, so the step's stores are non-temporal: they no longer evict from L2
// the side-halo lines that a strip's shifted pulls share with the
// neighbouring strip.  In FP64 the loads of the planes with e_x = 0, which
// no other strip touches, are non-temporal too, and the stores also carry
// sc1.  The choice per precision is measured (FP32 -7 %, FP64 -5 % step
// time on a 1024 x 2048 lattice; no change in FP16-dev).
template <int P> struct Policy { static constexpr int kStore = 2, kLoadOwn = 0; };
template <> struct Policy<P64> { static constexpr int kStore = 18, kLoadOwn = 2; };

// population k of family f at lattice node j (element offset within a plane);
// with `on` false the load is out of range: it returns 0 and touches no memory
template <int P>
__device__ __forceinline__ typename Tr<P>::R bld(const LatView<P>& v,
                                                 const Consts<typename Tr<P>::R>& c, int f,
                                                 int k, unsigned j, bool on) {
    if constexpr (P == P64) {
        const int vo = int(on ? j * 8u : kDiscard);
        auto r = EX[k] == 0
                     ? __builtin_amdgcn_raw_buffer_load_b64(v.fam[f], vo, int(k * v.pstride),
                                                            Policy<P>::kLoadOwn)
                     : __builtin_amdgcn_raw_buffer_load_b64(v.fam[f], vo, int(k * v.pstride), 0);
        return __builtin_bit_cast(double, r);
    } else if constexpr (P == P32) {
        unsigned r = __builtin_amdgcn_raw_buffer_load_b32(v.fam[f], int(on ? j * 4u : kDiscard),
                                                          int(k * v.pstride), 0);
        return __builtin_bit_cast(float, r);
    } else {
        // f^1_0, f^2_0 from the rest planes and the FP32 g planes here; the
        // f^1, f^2 pairs of k >= 1 are loaded together by bld12
        const unsigned r = __builtin_amdgcn_raw_buffer_load_b32(
            f < 2 ? v.rest : v.fam[2], int(on ? j * 4u : kDiscard),
            int(f < 2 ? f * v.rstride : k * v.pstride), 0);
        return __builtin_bit_cast(float, r);
    }
}

// store population k of family f at byte offset `ob` within its plane
// (`orb`: byte offset of a 4-byte element, for the FP32 rest and g planes of
// P16)
template <int P>
__device__ __forceinline__ void bst(const LatView<P>& v, const Consts<typename Tr<P>::R>& c,
                                    int f, int k, unsigned ob, unsigned orb,
                                    typename Tr<P>::R x) {
    if constexpr (P == P64) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(
            __builtin_amdgcn_raw_buffer_load_b64(v.fam[f], 0, 0, 0)), x), v.fam[f], int(ob),
            int(k * v.pstride), Policy<P>::kStore);
    } else if constexpr (P == P32) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), v.fam[f], int(ob),
                                              int(k * v.pstride), Policy<P>::kStore);
    } else {
        // f^1_0, f^2_0 to the rest planes and g to its FP32 planes; f^1, f^2
        // pairs of k >= 1 go through bst12
        (void)ob;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x),
                                              f < 2 ? v.rest : v.fam[2], int(orb),
                                              int(f < 2 ? f * v.rstride : k * v.pstride),
                                              Policy<P>::kStore);
    }
}

// f^1_k and f^2_k at node j together: one load of the pair word in P16.
// P16 keeps the moving populations (k >= 1) in registers in their stored,
// scaled form S_i f^i_k (S_i = c.scale[i], a power of two, so the scaling is
// exact): the step kernel folds S_i into its per-node collision terms and
// 1/S_i into the moment sums (sum_pop) instead of converting every
// population on load and on store.
template <int P>
__device__ __forceinline__ void bld12(const LatView<P>& v, const Consts<typename Tr<P>::R>& c,
                                      int k, unsigned j, bool on, typename Tr<P>::R& x1,
                                      typename Tr<P>::R& x2) {
    if constexpr (P == P16) {
        if (k > 0) {
            const unsigned r = __builtin_amdgcn_raw_buffer_load_b32(
                v.fam[(k - 1) >> 2], int(on ? j * 4u : kDiscard),
                int(unsigned((k - 1) & 3) * v.ppstride), 0);
            x1 = float(__builtin_bit_cast(_Float16, (unsigned short)(r & 0xffffu)));
            x2 = float(__builtin_bit_cast(_Float16, (unsigned short)(r >> 16)));
            return;
        }
    }
    x1 = bld<P>(v, c, 0, k, j, on);
    x2 = bld<P>(v, c, 1, k, j, on);
}

// store f^1_k and f^2_k of one node (byte offsets ob of an S element, o4 of a
// 4-byte element): one store of the pair word in P16, whose moving
// populations arrive already scaled (see bld12)
template <int P>
__device__ __forceinline__ void bst12(const LatView<P>& v, const Consts<typename Tr<P>::R>& c,
                                      int k, unsigned ob, unsigned o4, typename Tr<P>::R x1,
                                      typename Tr<P>::R x2) {
    if constexpr (P == P16) {
        if (k > 0) {
            const _Float16 h1 = _Float16(x1), h2 = _Float16(x2);
            const unsigned w = unsigned(__builtin_bit_cast(unsigned short, h1)) |
                               (unsigned(__builtin_bit_cast(unsigned short, h2)) << 16);
            __builtin_amdgcn_raw_buffer_store_b32(w, v.fam[(k - 1) >> 2], int(o4),
                                                  int(unsigned((k - 1) & 3) * v.ppstride),
                                                  Policy<P>::kStore);
            return;
        }
    }
    bst<P>(v, c, 0, k, ob, o4, x1);
    bst<P>(v, c, 1, k, ob, o4, x2);
}

// c_i = sum_k f^i_k (Eq. 13a) of the nine pulled populations of family i,
// in the order k = 0..8; in P16 the moving ones enter as S_i f^i_k times the
// exact factor 1/S_i
template <int P>
__device__ __forceinline__ typename Tr<P>::R sum_pop(const Consts<typename Tr<P>::R>& c, int i,
                                                     const typename Tr<P>::R* v) {
    typename Tr<P>::R a = v[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        if constexpr (P == P16)
            a = __builtin_fmaf(v[k], c.iscale[i], a);
        else
            a += v[k];
    }
    return a;
}

template <int P>
struct Ring {
    using R = typename Tr<P>::R;
    static constexpr int W = kTileX + 4;   // c ring columns x0-2 .. x0+65
    static constexpr int MW = kTileX + 2;  // mu ring columns x0-1 .. x0+64
    static constexpr int NR = 16;          // c ring rows (rows Y-1..Y+9 live at once)
    static constexpr int NM = 8;           // mu ring rows (rows Y-1..Y+4 live; a barrier
                                           // separates their last reader from the next writer)
    R c1[NR * W];
    R c2[NR * W];
    R mu1[NM * MW];
    R mu2[NM * MW];
    R mu3[NM * MW];
    R stash[2][2][18][kTileX];             // [buffer][wave-2][population][lane]
    R mt[kMatStride * (kMaxMaterials + 1)];
    uint32_t nmask[NM * MW];               // neighbour mask (kWallBits, kSelfBit, kVelBits)
    uint8_t m[NR * W];
};

__device__ __forceinline__ int ring_slot(int y, int y0) { return (y - y0 + 4) & 15; }
__device__ __forceinline__ int mu_slot(int y, int y0) { return (y - y0 + 4) & 7; }

// wrapped neighbourhood of (x, y) as 32-bit element offsets
struct Nb32 {
    unsigned xm, x0, xp, rm, r0, rp;
    __device__ __forceinline__ unsigned at(int dx, int dy) const {
        const unsigned r = dy < 0 ? rm : (dy > 0 ? rp : r0);
        const unsigned x = dx < 0 ? xm : (dx > 0 ? xp : x0);
        return r + x;
    }
    __device__ __forceinline__ unsigned up(int k) const { return at(-EX[k], -EY[k]); }
    __device__ __forceinline__ unsigned dn(int k) const { return at(EX[k], EY[k]); }
};

__device__ __forceinline__ Nb32 make_nb32(const Grid& g, int x, int y) {
    Nb32 n;
    n.x0 = unsigned(x);
    n.xm = unsigned(x == 0 ? g.nx - 1 : x - 1);
    n.xp = unsigned(x == g.nx - 1 ? 0 : x + 1);
    n.r0 = unsigned(y) * unsigned(g.pitch);
    n.rm = unsigned(y == 0 ? g.ny - 1 : y - 1) * unsigned(g.pitch);
    n.rp = unsigned(y == g.ny - 1 ? 0 : y + 1) * unsigned(g.pitch);
    return n;
}

// Issues the material byte and the 18 pulls of f^1, f^2 at node (gx, gy).
// The pulls are issued whatever the material (every wrapped offset is
// valid), so nothing waits on the byte before they go out; the values of a
// solid node are discarded where c is formed.  A row the strip does not need
// (`on` false) issues the same instructions out of range: no traffic, and
// the same wait pattern as every other iteration.
template <int P>
__device__ __forceinline__ void pull_f(const Grid& g, const Consts<typename Tr<P>::R>& c,
                                       const LatView<P>& src, rsrc_t mat,
                                       int gx, int gy, bool on, typename Tr<P>::R* f1,
                                       typename Tr<P>::R* f2, uint8_t& m) {
    const Nb32 nb = make_nb32(g, gx, gy);
    m = uint8_t(__builtin_amdgcn_raw_buffer_load_b8(mat, int(nb.r0 + nb.x0), 0, 0));
#pragma unroll
    for (int k = 0; k < 9; ++k) bld12<P>(src, c, k, nb.up(k), on, f1[k], f2[k]);
}

// Chemical potentials of one mu-ring node (mu column mcol, c column
// mcol + 1) and its solid-neighbour mask.
template <int P, unsigned F, class RG>
__device__ __forceinline__ void ring_mu(RG& sm, const typename Tr<P>::R* mt,
                                        const Consts<typename Tr<P>::R>& c, int y, int y0, int mcol) {
    using R = typename Tr<P>::R;
    const int sc[3] = {ring_slot(y - 1, y0), ring_slot(y, y0), ring_slot(y + 1, y0)};
    const int col = mcol + 1;
    const R* c1r[3];
    const R* c2r[3];
    const uint8_t* mr[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        c1r[q] = &sm.c1[sc[q] * RG::W + col];
        c2r[q] = &sm.c2[sc[q] * RG::W + col];
        mr[q] = &sm.m[sc[q] * RG::W + col];
    }
    // the whole 3x3 neighbourhood (material bytes and both c values) is read
    // before anything depends on it, so the LDS latency is paid once
    uint8_t mb[9];
    R v1[9], v2[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        mb[k] = mr[EY[k] + 1][EX[k]];
        v1[k] = c1r[EY[k] + 1][EX[k]];
        v2[k] = c2r[EY[k] + 1][EX[k]];
    }
    unsigned mask = mb[0] ? kSelfBit : 0u;
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        const unsigned mn = mb[k];
        if (mn)
            mask |= ((F & kFeatVel) && ((c.nee >> mn) & 1u)) ? 1u << (kVelShift + k) : 1u << (k - 1);
    }
    // the bulk form, plain Laplacian (Eq. 20b), is evaluated for every node
    // (so that the reads above stay ahead of the mask) and replaced where the
    // node is solid or has a solid neighbour
    R mu1, mu2, mu3;
    {
        const R a1 = v1[0], a2 = v2[0], a3 = R(1) - a1 - a2;
        R l1 = R(0), l2 = R(0);
#pragma unroll
        for (int k = 1; k < 9; ++k) {
            l1 += wgt<R>(k) * (v1[k] - a1);
            l2 += wgt<R>(k) * (v2[k] - a2);
        }
        l1 *= R(6);
        l2 *= R(6);
        const R l3 = -(l1 + l2);   // c3 = 1 - c1 - c2 at every node of the stencil
        const R tri = R(2) * c.lamT * a1 * a2 * (R(1) - a1 - a2);
        mu1 = c.k12D * (c.lam1 * a1 * (R(1) - a1) * (R(1) - R(2) * a1) - tri) - c.k34D * c.lam1 * l1;
        mu2 = c.k12D * (c.lam2 * a2 * (R(1) - a2) * (R(1) - R(2) * a2) - tri) - c.k34D * c.lam2 * l2;
        mu3 = c.k12D * (c.lam3 * a3 * (R(1) - a3) * (R(1) - R(2) * a3) - tri) - c.k34D * c.lam3 * l3;
        lambda_term<R, (F & kFeatLam) != 0>(c, a1, a2, mu1, mu2, mu3);
    }
    if (mask != 0) {
        if (mask & kSelfBit) {
            mu1 = mu2 = mu3 = R(0);
        } else {
            chem_pot<R, (F & kFeatVel) != 0, (F & kFeatLam) != 0>(c1r, c2r, mr, mt, c, mu1, mu2,
                                                                  mu3);
        }
    }
    const int o = mu_slot(y, y0) * RG::MW + mcol;
    sm.mu1[o] = mu1;
    sm.mu2[o] = mu2;
    sm.mu3[o] = mu3;
    sm.nmask[o] = mask;
}

// Where phase C puts a node's results in HBM: the node's own slots (byte
// offsets ob of an S element and o4 of a 4-byte element, both kDiscard for a
// lane without a fluid output node), slots of its neighbours, and the history
// planes.
template <int P>
struct HbmSink {
    using R = typename Tr<P>::R;
    using HT = typename Tr<P>::H;
    const LatView<P>& dst;
    const Consts<R>& c;
    rsrc_t hist;
    unsigned hstride;
    Nb32 nb;
    unsigned ob, o4;
    __device__ __forceinline__ void history(const HT (&hv)[4]) const {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (P == P64)
                __builtin_amdgcn_raw_buffer_store_b64(
                    __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(hist, 0, 0, 0)),
                                       hv[q]),
                    hist, int(ob), int(q * hstride), 0);
            else
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, hv[q]), hist,
                                                      int(o4), int(q * hstride), 0);
        }
    }
    // populations k of f^1, f^2 and g of the node
    __device__ __forceinline__ void own(int k, R x1, R x2, R gv) const {
        bst12<P>(dst, c, k, ob, o4, x1, x2);
        bst<P>(dst, c, 2, k, ob, o4, gv);
    }
    // populations q of the neighbour x + e_k
    __device__ __forceinline__ void link(int k, int q, R x1, R x2, R gv) const {
        const unsigned sn = nb.dn(k);
        const unsigned sb = sn * unsigned(sizeof(typename Tr<P>::S)), s4 = sn * 4u;
        bst12<P>(dst, c, q, sb, s4, x1, x2);
        bst<P>(dst, c, 2, q, sb, s4, gv);
    }
};

// Phase C of one node: time derivative (Eq. 19 in Eq. 11a), history,
// equilibria (Eqs. 2, 4), sources (Eq. 11), BGK collision (Eq. 45), the 27
// post-collision populations of the node (or nothing when `live` is false)
// and, for a node next to solids, half-way bounce-back into the solid slots
// (Eq. 44) with the moving-wall term -2 w_k a e_k.u_w / c_s^2 (a = c_i for
// f^i, rho for g); `out` stores them (HbmSink, or the LDS ring of the
// two-level march).
template <int P, unsigned F, class Sink>
__device__ __forceinline__ void node_update(const Consts<typename Tr<P>::R>& c,
                                            const Stencil<typename Tr<P>::R>& s,
                                            const typename Tr<P>::R* mt, bool live, unsigned mask,
                                            typename Tr<P>::R* f1, typename Tr<P>::R* f2,
                                            const typename Tr<P>::R* gg,
                                            const typename Tr<P>::R* ho, const Sink& out) {
    using R = typename Tr<P>::R;
    using HT = typename Tr<P>::H;
    constexpr bool VEL = (F & kFeatVel) != 0;
    const NodeMacro<R> o = node_macro<R, true, VEL>(s, c, gg, mask);
    const R d1x = o.c1 * o.ux - ho[0] * ho[2], d1y = o.c1 * o.uy - ho[0] * ho[3];
    const R d2x = o.c2 * o.ux - ho[1] * ho[2], d2y = o.c2 * o.uy - ho[1] * ho[3];
    {
        const HT hv[4] = {HT(o.c1), HT(o.c2), HT(o.ux), HT(o.uy)};
        out.history(hv);
    }
    // The collision of Eq. 45 with the equilibria of Eqs. 2 and 4 and the
    // sources of Eq. 11, regrouped into per-node scalars and vectors so that
    // each direction k costs a few fused operations:
    //   f'^i_k = (1 - 1/tau_i) f^i_k + w_k (P_i + e_k.V_i),  k != 0
    //   P_i = eta_i mu_i / tau_i,  V_i = 3 (c_i u / tau_i + (1 - 1/(2 tau_i)) D_i)
    //   g'_k = (1 - 1/tau_g) g_k + w_k (3 p / tau_g + e_k.G1 - G0)
    //          + s_k (rho / tau_g + fsg (e_k.A - u.A))
    //   A = grad rho + 3 (F_s + G),  G1 = 3 fsg (F_s + G) + 3 F_a,
    //   G0 = 3 fsg u.(F_s + G),  fsg = 1 - 1/(2 tau_g)
    const R uu = o.ux * o.ux + o.uy * o.uy;
    const R em1 = c.eta1 * o.mu1, em2 = c.eta2 * o.mu2;
    const R fsg = R(1) - R(0.5) * o.itg;
    const R om1 = R(1) - c.itau1, om2 = R(1) - c.itau2, omg = R(1) - o.itg;
    // P16: f1, f2 (k >= 1) hold S_i f^i_k, so every term added to them is
    // scaled by S_i too (exactly: S_i is a power of two)
    R S1 = R(1), S2 = R(1);
    if constexpr (P == P16) {
        S1 = c.scale[0];
        S2 = c.scale[1];
    }
    const R P1 = S1 * (c.itau1 * em1), P2 = S2 * (c.itau2 * em2);
    const R V1x = S1 * (R(3) * (c.itau1 * o.c1 * o.ux + c.fs1 * d1x));
    const R V1y = S1 * (R(3) * (c.itau1 * o.c1 * o.uy + c.fs1 * d1y));
    const R V2x = S2 * (R(3) * (c.itau2 * o.c2 * o.ux + c.fs2 * d2x));
    const R V2y = S2 * (R(3) * (c.itau2 * o.c2 * o.uy + c.fs2 * d2y));
    const R sc1 = S1 * o.c1, sc2 = S2 * o.c2;
    const R Ax = o.grx + R(3) * o.fx, Ay = o.gry + R(3) * o.fy;
    const R uA = o.ux * Ax + o.uy * Ay;
    const R G1x = R(3) * (fsg * o.fx + o.fax), G1y = R(3) * (fsg * o.fy + o.fay);
    const R G0 = R(3) * fsg * (o.ux * o.fx + o.uy * o.fy);
    const R Pg = R(3) * o.itg * o.p;
    const R Rg = o.itg * o.rho;
    // Velocity boundary node x_u = x + e_kn directly above (kn = 2) or below
    // (kn = 4) this node.  Its populations are its equilibrium plus this
    // node's non-equilibrium part (Eqs. 51-53): with every quantity but u
    // taken from this node, f^i_k(x_u) = f^i_k + 3 w_k c_i e_k.(u_w - u) and
    // g_k(x_u) = g_k + rho (s_k(u_w) - s_k(u)).  x_u collides like any node
    // (Eq. 45) with the sources of Eq. 11 at u = u_w: V_i and G1, G0 above
    // with u_w, D_i = u_w (c_i - c_i^old).  Only the three populations that
    // stream back into the fluid are stored.  Done before this node's own
    // stores so that nothing extra stays live across them.
    if (VEL && live && (mask & kVelBits)) {
#pragma unroll
        for (int kn = 2; kn <= 4; kn += 2) {
            if (!(mask & (1u << (kVelShift + kn)))) continue;
            const int mn = s.m[EY[kn] + 1][0];
            const R uwx = mt[kMatStride * mn + 3], uwy = mt[kMatStride * mn + 4];
            // e_k.V_i at u_w is 3 e_k.u_w a_i with a_i = c_i / tau_i + (1 - 1/(2 tau_i))
            // (c_i - c_i^old); e_k.G1 = 3 fsg e_k.F + 3 am e_k.u_w, G0 = 3 fsg u_w.F
            const R a1 = S1 * (c.itau1 * o.c1 + c.fs1 * (o.c1 - ho[0]));
            const R a2 = S2 * (c.itau2 * o.c2 + c.fs2 * (o.c2 - ho[1]));
            const R wF = uwx * o.fx + uwy * o.fy;
            const R wA = uwx * Ax + uwy * Ay;
            const R ww = uwx * uwx + uwy * uwy;
#pragma unroll
            for (int k = 1; k < 9; ++k) {
                if (EY[k] != -EY[kn]) continue;
                const R w = wgt<R>(k);
                const R eu = R(EX[k]) * o.ux + R(EY[k]) * o.uy;
                const R ew = R(EX[k]) * uwx + R(EY[k]) * uwy;
                const R sku = w * (eu * (R(3) + R(4.5) * eu) - R(1.5) * uu);
                const R skw = w * (ew * (R(3) + R(4.5) * ew) - R(1.5) * ww);
                const R eA = R(EX[k]) * Ax + R(EY[k]) * Ay;
                const R eF = R(EX[k]) * o.fx + R(EY[k]) * o.fy;
                const R f1u = om1 * (f1[k] + R(3) * w * sc1 * (ew - eu)) + w * (P1 + R(3) * ew * a1);
                const R f2u = om2 * (f2[k] + R(3) * w * sc2 * (ew - eu)) + w * (P2 + R(3) * ew * a2);
                const R gu = omg * (gg[k] + o.rho * (skw - sku)) +
                             w * (Pg + R(3) * (fsg * (eF - wF) + o.am * ew)) +
                             skw * (Rg + fsg * (eA - wA));
                out.link(kn, k, f1u, f2u, gu);
            }
        }
    }
    R g2[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const R w = wgt<R>(k);
        const R eu = R(EX[k]) * o.ux + R(EY[k]) * o.uy;
        const R sk = w * (eu * (R(3) + R(4.5) * eu) - R(1.5) * uu);       // Eq. 4
        if (k == 0) {
            f1[0] = om1 * f1[0] + c.itau1 * (o.c1 + (w - R(1)) * em1);
            f2[0] = om2 * f2[0] + c.itau2 * (o.c2 + (w - R(1)) * em2);
            g2[0] = omg * gg[0] + (w - R(1)) * Pg + sk * (Rg - fsg * uA) - w * G0;
        } else {
            const R eV1 = R(EX[k]) * V1x + R(EY[k]) * V1y;
            const R eV2 = R(EX[k]) * V2x + R(EY[k]) * V2y;
            const R eA = R(EX[k]) * Ax + R(EY[k]) * Ay;
            const R eG = R(EX[k]) * G1x + R(EY[k]) * G1y;
            f1[k] = om1 * f1[k] + w * (P1 + eV1);
            f2[k] = om2 * f2[k] + w * (P2 + eV2);
            g2[k] = omg * gg[k] + w * (Pg + eG - G0) + sk * (Rg + fsg * (eA - uA));
        }
        out.own(k, f1[k], f2[k], g2[k]);
    }
    if (live && (mask & kWallBits)) {
#pragma unroll
        for (int k = 1; k < 9; ++k) {
            if (mask & (1u << (k - 1))) {
                const int mn = s.m[EY[k] + 1][EX[k]];
                const R* tm = &mt[kMatStride * mn];
                const R corr = -R(6) * wgt<R>(k) * (R(EX[k]) * tm[3] + R(EY[k]) * tm[4]);
                out.link(k, OPP[k], f1[k] + corr * sc1, f2[k] + corr * sc2, g2[k] + corr * o.rho);
            }
        }
    }

}

// One strip (tile t) of one lattice.
template <int P, unsigned F>
__device__ __forceinline__ void step_tile(const Grid& g, const Consts<typename Tr<P>::R>& c,
                                          const uint8_t* __restrict__ mat,
                                          const double* __restrict__ mtab, PopBuf srcb,
                                          PopBuf dstb, typename Tr<P>::H* __restrict__ histp,
                                          int t, Ring<P>& sm) {
    using R = typename Tr<P>::R;
    using HT = typename Tr<P>::H;
    using RG = Ring<P>;
    const int x0 = (t % g.tiles_x) * kTileX;
    const int H = g.tile_rows;                             // strip height, a multiple of 4
    const int y0 = (t / g.tiles_x) * H;
    const int rows = g.ny - y0 < H ? g.ny - y0 : H;
    const int nit = (rows + 3) / 4;
    const int ylast = y0 + rows + 1;                       // last row whose c is needed
    const int lane = threadIdx.x & (kTileX - 1);
    const int w = threadIdx.x / kTileX;
    const LatView<P> src = lat_view<P>(srcb, g.npad);
    // Every memory access of the step goes through buffer resources or
    // global-space pointers: a pending generic (flat) load, which might touch
    // LDS, makes the compiler drain all outstanding loads at every wait.
    const rsrc_t matr = make_rsrc(mat, unsigned(g.npad));
    const auto* gmtab = (const __attribute__((address_space(1))) double*)mtab;
    for (int i = threadIdx.x; i < kMatStride * (kMaxMaterials + 1); i += kStepThreads)
        sm.mt[i] = R(gmtab[i]);

    // phase B of iteration it: mu on rows Y+1..Y+4, mu columns 0..65
    auto phase_b = [&](int it) {
        const int Y = y0 + 4 * it;
        if (threadIdx.x < 4 * RG::MW) {
            const int r = threadIdx.x / RG::MW;
            const int mcol = threadIdx.x - r * RG::MW;
            const int y = Y + 1 + r;
            if (y >= y0 - 1) ring_mu<P, F>(sm, sm.mt, c, y, y0, mcol);  // prologue: rows below y0-1 lack neighbours
        }
    };

    R nf1[9], nf2[9];
    uint8_t nm;
    if (w == 4) {
        // ---- halo wave: lanes 0..15 own node (row Y+2+(lane>>2), column
        //      x0-2, x0-1, x0+64, x0+65 for lane&3 = 0..3) of each iteration
        const int hc = lane & 3;
        const int ccol = hc < 2 ? hc : kTileX + hc;            // c ring column 0, 1, 66, 67
        const int gx = wrapc(x0 - 2 + ccol, g.nx);
        const int hr = (lane >> 2) & 3;
        const bool act = lane < 16;
        auto halo_a = [&](int it) {
            const int Y = y0 + 4 * it;
            const R a = sum_pop<P>(c, 0, nf1), b = sum_pop<P>(c, 1, nf2);
            if (act) {
                const int sl = ring_slot(Y + 2 + hr, y0) * RG::W + ccol;
                const bool fl = nm == 0;
                sm.c1[sl] = fl ? a : R(0);
                sm.c2[sl] = fl ? b : R(0);
                sm.m[sl] = nm;
            }
            pull_f<P>(g, c, src, matr, gx, wrapc(Y + 6 + hr, g.ny), act && Y + 6 + hr <= ylast,
                      nf1, nf2, nm);
        };
        pull_f<P>(g, c, src, matr, gx, wrapc(y0 - 2 + hr, g.ny), act, nf1, nf2, nm);
        halo_a(-1);
        __syncthreads();
        phase_b(-1);
        __syncthreads();
        halo_a(0);
        for (int it = 0; it < nit; ++it) {
            __syncthreads();
            phase_b(it);
            __syncthreads();
            halo_a(it + 1);
        }
        return;
    }

    // ---- row waves
    const int gxl = wrapc(x0 + lane, g.nx);                 // this lane's column
    const bool out_lane = x0 + lane < g.nx;
    const LatView<P> dst = lat_view<P>(dstb, g.npad);
    const unsigned hstride = unsigned(g.npad * long(sizeof(HT)));
    const rsrc_t hist = make_rsrc(histp, 4u * hstride);   // history, updated in place (Eq. 19)
    if constexpr (P == P64) {
        // Two register sets of pulled populations alternate (the loop is
        // unrolled by two): phase A of iteration it consumes the set pulled
        // one iteration earlier (u) and pulls the next row into the other
        // (f); phase C of iteration it uses u.  With one set carried around
        // the loop (the FP32 / FP16-dev code below), the FP64 kernel kept the
        // consumed copy in the loop-carried registers and moved the new pulls
        // into them at the back edge, which waits for every pull before the
        // barrier: 228 us per step against 215 us with two sets.  In FP32 and
        // FP16-dev a second set does not fit the 128-VGPR budget (spills;
        // FP32 111 -> 152 us), and the two-set source compiled to a 3 %
        // slower FP32 kernel even with the copy, so they keep the code below.
        R fb1[9], fb2[9], gg[9], ho[4];
        uint8_t mb;
        Nb32 nb;
        unsigned idx = 0;
        int yo = 0;

        // phase A of iteration it: c of row Y+2+w from the prefetched pulls u,
        // then the phase-C operands of iteration it (and, in the prologue, the
        // pulls for iteration 0 into f; later pulls are issued in phase C)
        auto phase_a = [&](int it, const R (&u1)[9], const R (&u2)[9], uint8_t um, R (&f1)[9],
                           R (&f2)[9], uint8_t& fm) {
            const int Y = y0 + 4 * it;
            const int sl = ring_slot(Y + 2 + w, y0) * RG::W + lane + 2;
            R a = R(0), b = R(0);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                a += u1[k];
                b += u2[k];
            }
            const bool fl = um == 0;
            sm.c1[sl] = fl ? a : R(0);
            sm.c2[sl] = fl ? b : R(0);
            sm.m[sl] = um;
            if (w >= 2) {
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    sm.stash[it & 1][w - 2][k][lane] = u1[k];
                    sm.stash[it & 1][w - 2][9 + k][lane] = u2[k];
                }
            }
            // issued on every path before the next row's pulls so that waiting
            // for them leaves those in flight; rows outside the strip load out of
            // range (no traffic)
            yo = Y + ((w + 2) & 3);
            nb = make_nb32(g, gxl, wrapc(yo, g.ny));
            idx = nb.r0 + nb.x0;
            const bool gon = yo >= y0 && yo < y0 + rows;
#pragma unroll
            for (int k = 0; k < 9; ++k) gg[k] = bld<P>(src, c, 2, k, nb.up(k), gon);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (P == P64)
                    ho[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                        hist, int(gon ? idx * 8u : kDiscard), int(q * hstride), 0));
                else
                    ho[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                        hist, int(gon ? idx * 4u : kDiscard), int(q * hstride), 0));
            }
            __builtin_amdgcn_sched_barrier(0);
            if (it < 0)
                pull_f<P>(g, c, src, matr, gxl, wrapc(Y + 6 + w, g.ny), Y + 6 + w <= ylast, f1, f2,
                          fm);
            __builtin_amdgcn_sched_barrier(0);
        };

        // phase C of iteration it: row wave w issues the pulls for iteration
        // it+1 into f, then updates row yo from u (waves 0, 1) or from the row
        // it parked in the stash one iteration earlier (waves 2, 3, loaded
        // into u, which phase A no longer needs)
        auto phase_c = [&](int it, R (&u1)[9], R (&u2)[9], R (&f1)[9], R (&f2)[9], uint8_t& fm) {
            Stencil<R> s;
            const int sl[3] = {ring_slot(yo - 1, y0), ring_slot(yo, y0), ring_slot(yo + 1, y0)};
            const int ml[3] = {mu_slot(yo - 1, y0), mu_slot(yo, y0), mu_slot(yo + 1, y0)};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                s.c1[r] = &sm.c1[sl[r] * RG::W + lane + 2];
                s.c2[r] = &sm.c2[sl[r] * RG::W + lane + 2];
                s.m[r] = &sm.m[sl[r] * RG::W + lane + 2];
                s.mu1[r] = &sm.mu1[ml[r] * RG::MW + lane + 1];
                s.mu2[r] = &sm.mu2[ml[r] * RG::MW + lane + 1];
            }
            s.mu3 = sm.mu3[ml[1] * RG::MW + lane + 1];
            const unsigned mask = out_lane ? sm.nmask[ml[1] * RG::MW + lane + 1] : kSelfBit;
            const bool live = out_lane && yo < y0 + rows && !(mask & kSelfBit);
            if (w >= 2) {
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    u1[k] = sm.stash[(it - 1) & 1][w - 2][k][lane];
                    u2[k] = sm.stash[(it - 1) & 1][w - 2][9 + k][lane];
                }
            }
            {
                const int Y = y0 + 4 * it;
                __builtin_amdgcn_sched_barrier(0);
                pull_f<P>(g, c, src, matr, gxl, wrapc(Y + 6 + w, g.ny), Y + 6 + w <= ylast, f1, f2,
                          fm);
                __builtin_amdgcn_sched_barrier(0);
            }
            const HbmSink<P> out{dst, c, hist, hstride, nb,
                                 live ? idx * unsigned(sizeof(typename Tr<P>::S)) : kDiscard,
                                 live ? idx * 4u : kDiscard};
            node_update<P, F>(c, s, sm.mt, live, mask, u1, u2, gg, ho, out);
        };

        pull_f<P>(g, c, src, matr, gxl, wrapc(y0 - 2 + w, g.ny), true, nf1, nf2, nm);
        // sets A (nf) and B (fb) alternate
        phase_a(-1, nf1, nf2, nm, fb1, fb2, mb);
        __syncthreads();
        phase_b(-1);
        __syncthreads();
        phase_a(0, fb1, fb2, mb, nf1, nf2, nm);
        for (int it = 0; it < nit; it += 2) {
            __syncthreads();
            phase_b(it);
            __syncthreads();
            phase_c(it, fb1, fb2, nf1, nf2, nm);
            // phase A of the next iteration (after the last one its loads
            // are all out of range)
            phase_a(it + 1, nf1, nf2, nm, fb1, fb2, mb);
            if (it + 1 == nit) break;
            __syncthreads();
            phase_b(it + 1);
            __syncthreads();
            phase_c(it + 1, nf1, nf2, fb1, fb2, mb);
            phase_a(it + 2, fb1, fb2, mb, nf1, nf2, nm);
        }
    } else {
        R cf1[9], cf2[9], gg[9], ho[4];
        Nb32 nb;
        unsigned idx = 0;
        int yo = 0;

        // phase A of iteration it: c of row Y+2+w from the prefetched pulls, then
        // the phase-C operands of iteration it.  The pulls for iteration it+1
        // are issued at the start of phase C (in the prologue, it = -1, here):
        // a row wave that issued them here, in one burst with the g / history
        // loads, stalled on issue while the other waves waited at the barrier
        // (FP32 111.7 -> 109.0 us per step on a 1024 x 2048 lattice).
        auto phase_a = [&](int it) {
            const int Y = y0 + 4 * it;
            const int sl = ring_slot(Y + 2 + w, y0) * RG::W + lane + 2;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                cf1[k] = nf1[k];
                cf2[k] = nf2[k];
            }
            const R a = sum_pop<P>(c, 0, cf1), b = sum_pop<P>(c, 1, cf2);
            const bool fl = nm == 0;
            sm.c1[sl] = fl ? a : R(0);
            sm.c2[sl] = fl ? b : R(0);
            sm.m[sl] = nm;
            if (w >= 2) {
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    sm.stash[it & 1][w - 2][k][lane] = cf1[k];
                    sm.stash[it & 1][w - 2][9 + k][lane] = cf2[k];
                }
            }
            // issued on every path before the next row's pulls so that waiting
            // for them leaves those in flight; rows outside the strip load out of
            // range (no traffic)
            yo = Y + ((w + 2) & 3);
            nb = make_nb32(g, gxl, wrapc(yo, g.ny));
            idx = nb.r0 + nb.x0;
            const bool gon = yo >= y0 && yo < y0 + rows;
#pragma unroll
            for (int k = 0; k < 9; ++k) gg[k] = bld<P>(src, c, 2, k, nb.up(k), gon);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (P == P64)
                    ho[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                        hist, int(gon ? idx * 8u : kDiscard), int(q * hstride), 0));
                else
                    ho[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                        hist, int(gon ? idx * 4u : kDiscard), int(q * hstride), 0));
            }
            __builtin_amdgcn_sched_barrier(0);
            if (it < 0)
                pull_f<P>(g, c, src, matr, gxl, wrapc(Y + 6 + w, g.ny), Y + 6 + w <= ylast, nf1, nf2,
                          nm);
            __builtin_amdgcn_sched_barrier(0);
        };

        pull_f<P>(g, c, src, matr, gxl, wrapc(y0 - 2 + w, g.ny), true, nf1, nf2, nm);
        phase_a(-1);
        __syncthreads();
        phase_b(-1);
        __syncthreads();
        phase_a(0);
        for (int it = 0; it < nit; ++it) {
            __syncthreads();
            phase_b(it);
            __syncthreads();
            // ---- phase C
            {
                Stencil<R> s;
                const int sl[3] = {ring_slot(yo - 1, y0), ring_slot(yo, y0), ring_slot(yo + 1, y0)};
                const int ml[3] = {mu_slot(yo - 1, y0), mu_slot(yo, y0), mu_slot(yo + 1, y0)};
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    s.c1[r] = &sm.c1[sl[r] * RG::W + lane + 2];
                    s.c2[r] = &sm.c2[sl[r] * RG::W + lane + 2];
                    s.m[r] = &sm.m[sl[r] * RG::W + lane + 2];
                    s.mu1[r] = &sm.mu1[ml[r] * RG::MW + lane + 1];
                    s.mu2[r] = &sm.mu2[ml[r] * RG::MW + lane + 1];
                }
                s.mu3 = sm.mu3[ml[1] * RG::MW + lane + 1];
                const unsigned mask = out_lane ? sm.nmask[ml[1] * RG::MW + lane + 1] : kSelfBit;
                const bool live = out_lane && yo < y0 + rows && !(mask & kSelfBit);
                if (w >= 2) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) {
                        cf1[k] = sm.stash[(it - 1) & 1][w - 2][k][lane];
                        cf2[k] = sm.stash[(it - 1) & 1][w - 2][9 + k][lane];
                    }
                }
                {
                    const int Y = y0 + 4 * it;
                    __builtin_amdgcn_sched_barrier(0);
                    pull_f<P>(g, c, src, matr, gxl, wrapc(Y + 6 + w, g.ny), Y + 6 + w <= ylast, nf1,
                              nf2, nm);
                    __builtin_amdgcn_sched_barrier(0);
                }
                const HbmSink<P> out{dst, c, hist, hstride, nb,
                                     live ? idx * unsigned(sizeof(typename Tr<P>::S)) : kDiscard,
                                     live ? idx * 4u : kDiscard};
                node_update<P, F>(c, s, sm.mt, live, mask, cf1, cf2, gg, ho, out);
            }
            // phase A of the next iteration (after the last one its loads are
            // all out of range)
            phase_a(it + 1);
        }
    }
}

// The step kernel: workgroups enumerate the strips of a table of lattices
// (one lattice, or a batch of independent lattices of any sizes and fluid
// parameters sharing one precision).  The table's tile_begin fields are the
// prefix sums of the lattices' strip counts; a workgroup finds its lattice by
// binary search.  parity selects which of each lattice's two population
// buffers is the source in this step.  A lattice's strips are computed by the
// same code whatever else is in the table, so results do not depend on the
// batch.  F (kFeatVel, kFeatLam) selects the optional parts that some
// lattice of the table needs.
template <int P, unsigned F>
__global__ __launch_bounds__(kStepThreads)
__attribute__((amdgpu_waves_per_eu(P == P64 ? 2 : 4)))
void step_kernel(const unsigned char* __restrict__ descs, int ndesc, int total_tiles, int parity) {
    using D = LatDesc<typename Tr<P>::R, typename Tr<P>::H>;
    // descriptors sit kDescBytes apart (not sizeof(D) apart)
    auto desc = [&](int i) -> const D& {
        return *reinterpret_cast<const D*>(descs + size_t(i) * kDescBytes);
    };
    __shared__ Ring<P> sm;
    const int L = tile_of(blockIdx.x, total_tiles);
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc(mid).tile_begin <= L) lo = mid;
        else hi = mid - 1;
    }
    const D& d = desc(lo);
    const Grid g = d.g;
    const Consts<typename Tr<P>::R> c = d.c;
    const int sb = (d.cur + parity) & 1;
    const int hb = (d.hcur ^ (parity >> 1)) & 1;
    step_tile<P, F>(g, c, d.mat, d.mtab, d.buf[sb], d.buf[sb ^ 1], d.hist[hb], L - d.tile_begin,
                    sm);
}

// ------------------------------------------------------------ two-step march
// step2_kernel advances a lattice by two time steps in one pass over its
// populations (FP32 storage; optional parts F as in step_kernel).  A
// workgroup of eleven waves marches a 64-column strip of rows [y0, y0 + H)
// at two time levels:
//   level 1 collides rows [y0-4, y0+H+4) and columns [x0-3, x0+67) from the
//     populations in HBM (the same phases as step_kernel) and keeps its
//     post-collision populations in an LDS ring of 8 rows (27 planes x 70
//     columns) instead of storing them;
//   level 2 trails level 1 by 8 rows, pulls from that ring, collides rows
//     [y0, y0+H) of columns [x0, x0+64) and stores to HBM.
// Level 2 is step_kernel's second step exactly: every node goes through the
// same pulls, moments, chemical potentials and collision (the same device
// functions), so two launches of step_kernel and one of step2_kernel give the
// same numbers.  Level 1 needs its own radius-3 frame (a node's c needs pulls
// from x +- 1, its mu the c of x +- 1, its collision the mu of x +- 1), hence
// 6 extra columns of collisions and 10 of c per 64 columns.
// Waves: 0-3 level-1 rows, 4 level-1 c on the 10 side columns, 5 level-1
// collisions on the 6 side columns, 6-9 level-2 rows, 10 level-2 c on the 4
// side columns.  Per iteration (four rows of each level) three barriers split
//   slot 1: level-1 mu (waves 0-4), the side waves' loads (4: the pulls of
//           their next c rows, 5: everything their collisions need) |
//           level-2 mu (waves 6-10);
//   slot 2: level-1 collisions into the ring (waves 0-3, 5) | level-2
//           collisions to HBM (waves 6-9), so that the nine colliding waves
//           share the SIMDs at once;
//   slot 3: level-1 c of the next rows and the g / history loads of the row
//           waves (waves 0-4) | level-2 c of the next rows from the ring
//           (waves 6-10).
// Level 2 reads ring rows only after the barrier that follows their level-1
// collision, and a ring slot is rewritten only after its last reader (see
// the row arithmetic at step2_tile).  Measured on a 1024 x 2048 lattice:
// with two slots (level-2 collision and c in one, level-1 collision in the
// other) the levels' collisions ran one after the other, 98.6 against
// 85.8 us per step; the side waves' loads in slot 3 made it the longer slot
// (85.8 against 81.4 us with them in slot 1).
// History planes: level 1 reads the history of the launch's input state and
// passes its own (c, u) to level 2 through an LDS ring; level 2 writes the
// output history to the other history set (another strip's level 1 may
// still read the input one).
constexpr int kStep2Waves = 11;
constexpr int kStep2Threads = kStep2Waves * kTileX;

template <int P>
struct Ring2 {
    using R = typename Tr<P>::R;
    static constexpr int PW = kTileX + 6;   // population ring columns x0-3 .. x0+66
    static constexpr int PS = PW + 1;       // row stride: column PW takes discarded stores
    static constexpr int PR = 8;            // population / history ring rows
    // c and mu rings of one level: c on columns x0-HC .. x0+63+HC, mu on one
    // column fewer each side (the layout ring_mu expects)
    template <int HC>
    struct Lvl {
        static constexpr int W = kTileX + 2 * HC, MW = kTileX + 2 * HC - 2;
        R c1[16 * W];
        R c2[16 * W];
        R mu1[8 * MW];
        R mu2[8 * MW];
        R mu3[8 * MW];
        uint32_t nmask[8 * MW];
        uint8_t m[16 * W];
    };
    R pop[27][PR][PS];                       // level-1 post-collision populations
    R stash1[2][2][18][kTileX];              // level-1 waves 2, 3 (as in Ring)
    R stash2[2][2][27][kTileX];              // level-2 waves 2, 3
    R hist[PR + 1][4][kTileX];               // level-1 (c1, c2, ux, uy) for level 2; row PR
                                             // takes discarded stores
    R mt[kMatStride * (kMaxMaterials + 1)];
    Lvl<5> a;                                // level 1
    Lvl<2> b;                                // level 2
};

// ring row of a population / history row y of a strip whose level 1 starts
// at row yb1 (rows yb1-1 .. are written)
__device__ __forceinline__ int pop_slot(int y, int yb1) { return (y - yb1 + 8) & 7; }

// Level-1 destination of a node's results: its column `col` (PW when the
// node is not live: the discard column) and row slot `rs` of the population
// ring, bounce-back into the ring's neighbour slots (to the discard column
// outside the ring's columns: no level-2 node pulls them), and its history
// (`hist`: its slot in the history ring, or in the discard row).  No store
// is behind a branch, so node_update compiles to the same arithmetic as with
// HbmSink.
template <int P>
struct LdsSink {
    using R = typename Tr<P>::R;
    using HT = typename Tr<P>::H;
    using RG = Ring2<P>;
    R* pop;
    R* hist;
    int rs, col;
    __device__ __forceinline__ void history(const HT (&hv)[4]) const {
#pragma unroll
        for (int q = 0; q < 4; ++q) hist[q * kTileX] = hv[q];
    }
    __device__ __forceinline__ void own(int k, R x1, R x2, R gv) const {
        pop[(k * RG::PR + rs) * RG::PS + col] = x1;
        pop[((9 + k) * RG::PR + rs) * RG::PS + col] = x2;
        pop[((18 + k) * RG::PR + rs) * RG::PS + col] = gv;
    }
    __device__ __forceinline__ void link(int k, int q, R x1, R x2, R gv) const {
        const int r = (rs + EY[k]) & (RG::PR - 1);
        const int c0 = col + EX[k];
        const int cc = unsigned(c0) < unsigned(RG::PW) ? c0 : RG::PW;
        pop[(q * RG::PR + r) * RG::PS + cc] = x1;
        pop[((9 + q) * RG::PR + r) * RG::PS + cc] = x2;
        pop[((18 + q) * RG::PR + r) * RG::PS + cc] = gv;
    }
};

// One strip of one lattice, two steps.  Rows: level 1 is step_tile's march
// with base yb1 = y0 - 4 and rows + 8 rows (iterations it = -1 .. nit2 + 1,
// Y1 = yb1 + 4 it); level 2 is the same march with base y0 (iterations
// j = -1 .. nit2 - 1, Y2 = y0 + 4 j).  At loop index it: slot 1 level-1 mu
// of it and level-2 mu of j = it - 3; slot 2 the collisions of level 1 (it)
// and level 2 (j = it - 3, Y2 = Y1 - 8); slot 3 level-1 c of it + 1 and
// level-2 c of j = it - 2.  Level-2 c of j = it - 2 pulls ring rows
// Y2+1 .. Y2+6 = Y1-3 .. Y1+2, collided by level 1 in slot 2 of this or an
// earlier index (rows <= Y1 + 3; later collisions write no row below Y1 + 3,
// their bounce-back included).
// Level-1 collision it writes rows Y1-1 .. Y1+4, whose slots (mod 8) held
// rows Y1-9 .. Y1-4, last read in slot 3 of index it - 1; the rows read in
// slot 3 of index it (Y1-3 .. Y1+2) are not among them.  The history ring
// row of a level-2 collision row is read with that row's c (slot 3, one
// index before the collision), before level 1 rewrites it in slot 2.
template <int P, unsigned F>
__device__ __forceinline__ void step2_tile(const Grid& g, int H, const Consts<typename Tr<P>::R>& c,
                                           const uint8_t* __restrict__ mat,
                                           const double* __restrict__ mtab, PopBuf srcb,
                                           PopBuf dstb, const typename Tr<P>::H* __restrict__ histi,
                                           typename Tr<P>::H* __restrict__ histo, int t,
                                           Ring2<P>& sm) {
    static_assert(P == P32, "the two-step march keeps FP32 populations in LDS");
    using R = typename Tr<P>::R;
    using HT = typename Tr<P>::H;
    using RG = Ring2<P>;
    using LA = typename RG::template Lvl<5>;
    using LB = typename RG::template Lvl<2>;
    const int x0 = (t % g.tiles_x) * kTileX;
    const int y0 = (t / g.tiles_x) * H;
    const int rows = g.ny - y0 < H ? g.ny - y0 : H;
    const int nit2 = (rows + 3) / 4;
    const int yb1 = y0 - 4, rows1 = rows + 8;
    const int nit1 = nit2 + 2;
    const int ylast1 = yb1 + rows1 + 1;                    // last level-1 row whose c is needed
    const int lane = threadIdx.x & (kTileX - 1);
    const int w = threadIdx.x / kTileX;
    const LatView<P> src = lat_view<P>(srcb, g.npad);
    const rsrc_t matr = make_rsrc(mat, unsigned(g.npad));
    const auto* gmtab = (const __attribute__((address_space(1))) double*)mtab;
    for (int i = threadIdx.x; i < kMatStride * (kMaxMaterials + 1); i += kStep2Threads)
        sm.mt[i] = R(gmtab[i]);
    const unsigned hstride = unsigned(g.npad * long(sizeof(HT)));
    const rsrc_t hist_in = make_rsrc(histi, 4u * hstride);
    const int itmax = nit2 + 2;

    // level-1 mu of iteration it (rows Y1+1 .. Y1+4, mu columns 0..71):
    // threads 0..287; level-2 mu of iteration j (rows Y2+1 .. Y2+4, columns
    // 0..65): threads 384..647
    auto b1 = [&](int it) {
        if (threadIdx.x < 4 * LA::MW) {
            const int r = threadIdx.x / LA::MW;
            const int mcol = threadIdx.x - r * LA::MW;
            const int y = yb1 + 4 * it + 1 + r;
            if (y >= yb1 - 1) ring_mu<P, F>(sm.a, sm.mt, c, y, yb1, mcol);
        }
    };
    auto b2 = [&](int j) {
        const int tt = int(threadIdx.x) - 6 * kTileX;
        if (tt >= 0 && tt < 4 * LB::MW) {
            const int r = tt / LB::MW;
            const int mcol = tt - r * LB::MW;
            const int y = y0 + 4 * j + 1 + r;
            if (y >= y0 - 1) ring_mu<P, F>(sm.b, sm.mt, c, y, y0, mcol);
        }
    };

    if (w < 6) {
        // ================================ level 1 (HBM -> ring)
        R nf1[9], nf2[9];
        uint8_t nm;
        if (w == 4) {
            // c of the 10 side columns x0-5 .. x0-1, x0+64 .. x0+68 (c ring
            // columns 0..4, 69..73), lane = column + 10 * (row - Y1 - 2)
            const int hc = lane % 10;
            const int hr = lane / 10;
            const bool act = lane < 40;
            const int ccol = hc < 5 ? hc : kTileX + hc;
            const int gx = wrapc(x0 - 5 + ccol, g.nx);
            auto halo_c = [&](int it) {
                const int Y = yb1 + 4 * it;
                const R a = sum_pop<P>(c, 0, nf1), b = sum_pop<P>(c, 1, nf2);
                if (act) {
                    const int sl = ring_slot(Y + 2 + hr, yb1) * LA::W + ccol;
                    const bool fl = nm == 0;
                    sm.a.c1[sl] = fl ? a : R(0);
                    sm.a.c2[sl] = fl ? b : R(0);
                    sm.a.m[sl] = nm;
                }
            };
            // pulls for the c rows of iteration it
            auto halo_pull = [&](int it) {
                const int Y = yb1 + 4 * it;
                pull_f<P>(g, c, src, matr, gx, wrapc(Y + 2 + hr, g.ny), act && Y + 2 + hr <= ylast1,
                          nf1, nf2, nm);
            };
            halo_pull(-1);
            halo_c(-1);
            for (int it = -1; it <= itmax; ++it) {
                __syncthreads();
                if (it <= nit1 - 1) b1(it);
                // pulls for the c rows of it + 1, formed in slot 3
                if (it + 1 <= nit1 - 1) halo_pull(it + 1);
                __syncthreads();
                __syncthreads();
                if (it + 1 <= nit1 - 1) halo_c(it + 1);
            }
            return;
        }
        if (w == 5) {
            // collisions of the 6 side columns x0-3 .. x0-1, x0+64 .. x0+66
            // (ring columns 0..2, 67..69), lane = column + 6 * (row - Y1);
            // their pulls, g and history are loaded in slot 1, one slot ahead
            const int hc = lane % 6;
            const int hr = lane / 6;
            const bool act = lane < 24;
            const int pcol = hc < 3 ? hc : kTileX + hc;
            const int gx = wrapc(x0 - 3 + pcol, g.nx);
            R gg[9], ho[4];
            Nb32 nb;
            auto side_a = [&](int it) {
                const int yo = yb1 + 4 * it + hr;
                const bool on = act && yo < yb1 + rows1;
                pull_f<P>(g, c, src, matr, gx, wrapc(yo, g.ny), on, nf1, nf2, nm);
                nb = make_nb32(g, gx, wrapc(yo, g.ny));
                const unsigned idx = nb.r0 + nb.x0;
#pragma unroll
                for (int k = 0; k < 9; ++k) gg[k] = bld<P>(src, c, 2, k, nb.up(k), on);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    ho[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                        hist_in, int(on ? idx * 4u : kDiscard), int(q * hstride), 0));
            };
            auto side_c = [&](int it) {
                const int yo = yb1 + 4 * it + hr;
                Stencil<R> s;
                const int sl[3] = {ring_slot(yo - 1, yb1), ring_slot(yo, yb1), ring_slot(yo + 1, yb1)};
                const int ml[3] = {mu_slot(yo - 1, yb1), mu_slot(yo, yb1), mu_slot(yo + 1, yb1)};
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    s.c1[r] = &sm.a.c1[sl[r] * LA::W + pcol + 2];
                    s.c2[r] = &sm.a.c2[sl[r] * LA::W + pcol + 2];
                    s.m[r] = &sm.a.m[sl[r] * LA::W + pcol + 2];
                    s.mu1[r] = &sm.a.mu1[ml[r] * LA::MW + pcol + 1];
                    s.mu2[r] = &sm.a.mu2[ml[r] * LA::MW + pcol + 1];
                }
                s.mu3 = sm.a.mu3[ml[1] * LA::MW + pcol + 1];
                const unsigned mask = act ? sm.a.nmask[ml[1] * LA::MW + pcol + 1] : kSelfBit;
                const bool live = act && yo < yb1 + rows1 && !(mask & kSelfBit);
                const LdsSink<P> out{&sm.pop[0][0][0], &sm.hist[RG::PR][0][lane], pop_slot(yo, yb1),
                                     live ? pcol : RG::PW};
                node_update<P, F>(c, s, sm.mt, live, mask, nf1, nf2, gg, ho, out);
            };
            for (int it = -1; it <= itmax; ++it) {
                __syncthreads();
                if (it >= 0 && it <= nit1 - 1) side_a(it);
                __syncthreads();
                if (it >= 0 && it <= nit1 - 1) side_c(it);
                __syncthreads();
            }
            return;
        }

        // ---- level-1 row waves: columns x0 .. x0+63 (c ring column lane+5,
        //      mu column lane+4, population ring column lane+3).  In a last
        //      strip narrower than 64 columns the lanes past nx step the
        //      wrapped columns 0, 1, 2, ..., which are that strip's right frame.
        const int gxl = wrapc(x0 + lane, g.nx);
        R cf1[9], cf2[9], gg[9], ho[4];
        int yo = 0;
        auto phase_a = [&](int it) {
            const int Y = yb1 + 4 * it;
            const int sl = ring_slot(Y + 2 + w, yb1) * LA::W + lane + 5;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                cf1[k] = nf1[k];
                cf2[k] = nf2[k];
            }
            const R a = sum_pop<P>(c, 0, cf1), b = sum_pop<P>(c, 1, cf2);
            const bool fl = nm == 0;
            sm.a.c1[sl] = fl ? a : R(0);
            sm.a.c2[sl] = fl ? b : R(0);
            sm.a.m[sl] = nm;
            if (w >= 2) {
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    sm.stash1[it & 1][w - 2][k][lane] = cf1[k];
                    sm.stash1[it & 1][w - 2][9 + k][lane] = cf2[k];
                }
            }
            yo = Y + ((w + 2) & 3);
            const Nb32 nb = make_nb32(g, gxl, wrapc(yo, g.ny));
            const unsigned idx = nb.r0 + nb.x0;
            const bool gon = yo >= yb1 && yo < yb1 + rows1;
#pragma unroll
            for (int k = 0; k < 9; ++k) gg[k] = bld<P>(src, c, 2, k, nb.up(k), gon);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                ho[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                    hist_in, int(gon ? idx * 4u : kDiscard), int(q * hstride), 0));
            __builtin_amdgcn_sched_barrier(0);
            if (it < 0)
                pull_f<P>(g, c, src, matr, gxl, wrapc(Y + 6 + w, g.ny), Y + 6 + w <= ylast1, nf1,
                          nf2, nm);
            __builtin_amdgcn_sched_barrier(0);
        };
        auto phase_c = [&](int it) {
            Stencil<R> s;
            const int sl[3] = {ring_slot(yo - 1, yb1), ring_slot(yo, yb1), ring_slot(yo + 1, yb1)};
            const int ml[3] = {mu_slot(yo - 1, yb1), mu_slot(yo, yb1), mu_slot(yo + 1, yb1)};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                s.c1[r] = &sm.a.c1[sl[r] * LA::W + lane + 5];
                s.c2[r] = &sm.a.c2[sl[r] * LA::W + lane + 5];
                s.m[r] = &sm.a.m[sl[r] * LA::W + lane + 5];
                s.mu1[r] = &sm.a.mu1[ml[r] * LA::MW + lane + 4];
                s.mu2[r] = &sm.a.mu2[ml[r] * LA::MW + lane + 4];
            }
            s.mu3 = sm.a.mu3[ml[1] * LA::MW + lane + 4];
            const unsigned mask = sm.a.nmask[ml[1] * LA::MW + lane + 4];
            const bool live = yo < yb1 + rows1 && !(mask & kSelfBit);
            if (w >= 2) {
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    cf1[k] = sm.stash1[(it - 1) & 1][w - 2][k][lane];
                    cf2[k] = sm.stash1[(it - 1) & 1][w - 2][9 + k][lane];
                }
            }
            {
                const int Y = yb1 + 4 * it;
                __builtin_amdgcn_sched_barrier(0);
                pull_f<P>(g, c, src, matr, gxl, wrapc(Y + 6 + w, g.ny), Y + 6 + w <= ylast1, nf1,
                          nf2, nm);
                __builtin_amdgcn_sched_barrier(0);
            }
            const int ps = pop_slot(yo, yb1);
            const LdsSink<P> out{&sm.pop[0][0][0], &sm.hist[live ? ps : RG::PR][0][lane], ps,
                                 live ? lane + 3 : RG::PW};
            node_update<P, F>(c, s, sm.mt, live, mask, cf1, cf2, gg, ho, out);
        };
        pull_f<P>(g, c, src, matr, gxl, wrapc(yb1 - 2 + w, g.ny), true, nf1, nf2, nm);
        phase_a(-1);
        for (int it = -1; it <= itmax; ++it) {
            __syncthreads();
            if (it <= nit1 - 1) b1(it);
            __syncthreads();
            if (it >= 0 && it <= nit1 - 1) phase_c(it);
            __syncthreads();
            if (it + 1 <= nit1 - 1) phase_a(it + 1);
        }
        return;
    }

    // ==================================== level 2 (ring -> HBM)
    const LatView<P> dst = lat_view<P>(dstb, g.npad);
    const rsrc_t hist_out = make_rsrc(histo, 4u * hstride);
    // pull of the 18 (or, with g, 27) populations of node (column pc of the
    // population ring + 0, row y) from the ring: plane q of x - e_k
    auto ring_pull = [&](int pc, int y, R* f1, R* f2, R* gv) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int r = pop_slot(y - EY[k], yb1);
            const int cc = pc - EX[k];
            f1[k] = sm.pop[k][r][cc];
            f2[k] = sm.pop[9 + k][r][cc];
            if (gv) gv[k] = sm.pop[18 + k][r][cc];
        }
    };
    if (w == 10) {
        // c of the 4 side columns x0-2, x0-1, x0+64, x0+65 (c ring columns
        // 0, 1, 66, 67), lane = column + 4 * (row - Y2 - 2)
        const int hc = lane & 3;
        const int hr = (lane >> 2) & 3;
        const bool act = lane < 16;
        const int ccol = hc < 2 ? hc : kTileX + hc;
        auto halo_a2 = [&](int j) {
            const int y = y0 + 4 * j + 2 + hr;
            R f1[9], f2[9];
            ring_pull(ccol + 1, y, f1, f2, nullptr);
            const uint8_t m = sm.a.m[ring_slot(y, yb1) * LA::W + ccol + 3];
            const R a = sum_pop<P>(c, 0, f1), b = sum_pop<P>(c, 1, f2);
            if (act) {
                const int sl = ring_slot(y, y0) * LB::W + ccol;
                const bool fl = m == 0;
                sm.b.c1[sl] = fl ? a : R(0);
                sm.b.c2[sl] = fl ? b : R(0);
                sm.b.m[sl] = m;
            }
        };
        for (int it = -1; it <= itmax; ++it) {
            __syncthreads();
            if (it - 3 >= -1 && it - 3 <= nit2 - 1) b2(it - 3);
            __syncthreads();
            __syncthreads();
            if (it - 2 >= -1 && it - 2 <= nit2 - 1) halo_a2(it - 2);
        }
        return;
    }

    // ---- level-2 row waves v = 0..3: c of row Y2+2+v, collision of row
    //      Y2 + ((v+2) & 3) (as step_tile's row waves)
    const int v = w - 6;
    const int gxl = wrapc(x0 + lane, g.nx);
    const bool out_lane = x0 + lane < g.nx;     // lanes past nx store nothing
    R p1[9], p2[9], pg[9], ho[4];
    auto a2 = [&](int j) {
        const int Z = y0 + 4 * j;
        const int y = Z + 2 + v;
        ring_pull(lane + 3, y, p1, p2, pg);
        const uint8_t m = sm.a.m[ring_slot(y, yb1) * LA::W + lane + 5];
        const R a = sum_pop<P>(c, 0, p1), b = sum_pop<P>(c, 1, p2);
        const int sl = ring_slot(y, y0) * LB::W + lane + 2;
        const bool fl = m == 0;
        sm.b.c1[sl] = fl ? a : R(0);
        sm.b.c2[sl] = fl ? b : R(0);
        sm.b.m[sl] = m;
        if (v >= 2) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                sm.stash2[j & 1][v - 2][k][lane] = p1[k];
                sm.stash2[j & 1][v - 2][9 + k][lane] = p2[k];
                sm.stash2[j & 1][v - 2][18 + k][lane] = pg[k];
            }
        }
        // history of the collision row of iteration j (read before level 1
        // reuses its ring row)
        const int yo = Z + ((v + 2) & 3);
#pragma unroll
        for (int q = 0; q < 4; ++q) ho[q] = sm.hist[pop_slot(yo, yb1)][q][lane];
    };
    auto c2 = [&](int j) {
        const int yo = y0 + 4 * j + ((v + 2) & 3);
        Stencil<R> s;
        const int sl[3] = {ring_slot(yo - 1, y0), ring_slot(yo, y0), ring_slot(yo + 1, y0)};
        const int ml[3] = {mu_slot(yo - 1, y0), mu_slot(yo, y0), mu_slot(yo + 1, y0)};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            s.c1[r] = &sm.b.c1[sl[r] * LB::W + lane + 2];
            s.c2[r] = &sm.b.c2[sl[r] * LB::W + lane + 2];
            s.m[r] = &sm.b.m[sl[r] * LB::W + lane + 2];
            s.mu1[r] = &sm.b.mu1[ml[r] * LB::MW + lane + 1];
            s.mu2[r] = &sm.b.mu2[ml[r] * LB::MW + lane + 1];
        }
        s.mu3 = sm.b.mu3[ml[1] * LB::MW + lane + 1];
        const unsigned mask = sm.b.nmask[ml[1] * LB::MW + lane + 1];
        const bool live = yo < y0 + rows && out_lane && !(mask & kSelfBit);
        if (v >= 2) {
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                p1[k] = sm.stash2[(j - 1) & 1][v - 2][k][lane];
                p2[k] = sm.stash2[(j - 1) & 1][v - 2][9 + k][lane];
                pg[k] = sm.stash2[(j - 1) & 1][v - 2][18 + k][lane];
            }
        }
        const Nb32 nb = make_nb32(g, gxl, wrapc(yo, g.ny));
        const unsigned idx = nb.r0 + nb.x0;
        const HbmSink<P> out{dst, c, hist_out, hstride, nb, live ? idx * 4u : kDiscard,
                             live ? idx * 4u : kDiscard};
        node_update<P, F>(c, s, sm.mt, live, mask, p1, p2, pg, ho, out);
    };
    for (int it = -1; it <= itmax; ++it) {
        __syncthreads();
        if (it - 3 >= -1 && it - 3 <= nit2 - 1) b2(it - 3);
        __syncthreads();
        if (it - 3 >= 0 && it - 3 <= nit2 - 1) c2(it - 3);
        __syncthreads();
        if (it - 2 >= -1 && it - 2 <= nit2 - 1) a2(it - 2);
    }
}

// Two steps per launch for a table of lattices (one, or a batch): a
// workgroup finds its lattice by binary search over the prefix-summed
// two-step strip counts, as step_kernel does over its own strips; parity
// selects the source buffer and history set as in step_kernel, and the
// result lands in the other ones.
template <int P, unsigned F>
__global__ __launch_bounds__(kStep2Threads)
void step2_kernel(const unsigned char* __restrict__ descs, int ndesc, int total_tiles,
                  int parity) {
    using D = LatDesc<typename Tr<P>::R, typename Tr<P>::H>;
    auto desc = [&](int i) -> const D& {
        return *reinterpret_cast<const D*>(descs + size_t(i) * kDescBytes);
    };
    __shared__ Ring2<P> sm;
    const int L = tile_of(blockIdx.x, total_tiles);
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc(mid).pair_tile_begin <= L) lo = mid;
        else hi = mid - 1;
    }
    const D& d = desc(lo);
    const Grid g = d.g;
    const Consts<typename Tr<P>::R> c = d.c;
    const int sb = (d.cur + parity) & 1;
    const int hb = (d.hcur ^ (parity >> 1)) & 1;
    step2_tile<P, F>(g, d.pair_rows, c, d.mat, d.mtab, d.buf[sb], d.buf[sb ^ 1], d.hist[hb],
                     d.hist[hb ^ 1], L - d.pair_tile_begin, sm);
}

// ------------------------------------------------------------------- init
// Equilibrium start (p = 0): writes f^eq(x) into the slots that x pulls
// from, history := (c1, c2, u0).
template <int P, int TY>
__global__ __launch_bounds__(kThreads) void init_kernel(Grid g, Consts<typename Tr<P>::R> c,
                                                        const uint8_t* __restrict__ mat,
                                                        const double* __restrict__ mtab,
                                                        const double* __restrict__ in4,
                                                        PopBuf dst,
                                                        typename Tr<P>::H* __restrict__ hist) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    __shared__ SM sm;
    const int t = blockIdx.x;
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    const int x0 = (t % ntx) * kTileX;
    const int y0 = (t / ntx) * TY;
    load_mtab<P, TY>(sm, mtab);
    phase_a<P, TY, false>(sm, g, c, mat, PopBuf{nullptr, nullptr}, in4, x0, y0);
    __syncthreads();
    phase_b<P, TY>(sm, c);
    __syncthreads();
    const int tx = threadIdx.x & (kTileX - 1);
    const int gx = x0 + tx;
    if (gx >= g.nx) return;
    const long n = long(g.nx) * g.ny;
    for (int ty = threadIdx.x / kTileX; ty < TY; ty += kThreads / kTileX) {
        const int gy = y0 + ty;
        if (gy >= g.ny) break;
        const int ci = (ty + 2) * SM::CW + tx + 2;
        const int mi = (ty + 1) * SM::MW + tx + 1;
        const Nb nb = make_nb(g, gx, gy);
        const long idx = nb.r0 + gx;
        const long hi = long(gy) * g.nx + gx;
        if (sm.m[ci]) {
#pragma unroll
            for (int q = 0; q < 4; ++q) hist[q * g.npad + idx] = typename Tr<P>::H(0);
            continue;
        }
        const R c1 = sm.c1[ci], c2 = sm.c2[ci];
        const R ux = R(in4[2 * n + hi]), uy = R(in4[3 * n + hi]);
        const R rho = c.rho3 + c.drho1 * c1 + c.drho2 * c2;
        const R em1 = c.eta1 * sm.mu1[mi], em2 = c.eta2 * sm.mu2[mi];
        const R uu = ux * ux + uy * uy;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const R w = wgt<R>(k);
            const R eu = R(EX[k]) * ux + R(EY[k]) * uy;
            const R sk = w * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
            R fe1, fe2;
            if (k == 0) {
                fe1 = c1 + (w - R(1)) * em1;
                fe2 = c2 + (w - R(1)) * em2;
            } else {
                fe1 = w * (em1 + R(3) * c1 * eu);
                fe2 = w * (em2 + R(3) * c2 * eu);
            }
            const R ge = rho * sk;
            const long j = nb.up(k);
            st<P>(dst, c, k, g.npad, j, fe1);
            st<P>(dst, c, 9 + k, g.npad, j, fe2);
            st<P>(dst, c, 18 + k, g.npad, j, ge);
        }
        hist[idx] = typename Tr<P>::H(c1);
        hist[g.npad + idx] = typename Tr<P>::H(c2);
        hist[2 * g.npad + idx] = typename Tr<P>::H(ux);
        hist[3 * g.npad + idx] = typename Tr<P>::H(uy);
    }
}

// ---------------------------------------------------------------- readout
template <int P, int TY>
__global__ __launch_bounds__(kThreads) void readout_kernel(Grid g, Consts<typename Tr<P>::R> c,
                                                           const uint8_t* __restrict__ mat,
                                                           const double* __restrict__ mtab,
                                                           PopBuf src, int ya, int yb,
                                                           double* __restrict__ out) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    __shared__ SM sm;
    const int t = blockIdx.x;
    const int ntx = (g.nx + kTileX - 1) / kTileX;
    const int x0 = (t % ntx) * kTileX;
    const int y0 = ya + (t / ntx) * TY;
    load_mtab<P, TY>(sm, mtab);
    phase_a<P, TY, true>(sm, g, c, mat, src, nullptr, x0, y0);
    __syncthreads();
    phase_b<P, TY>(sm, c);
    __syncthreads();
    const int tx = threadIdx.x & (kTileX - 1);
    const int gx = x0 + tx;
    if (gx >= g.nx) return;
    const long n = long(g.nx) * (yb - ya);               // nodes of the band
    for (int ty = threadIdx.x / kTileX; ty < TY; ty += kThreads / kTileX) {
        const int gy = y0 + ty;
        if (gy >= yb) break;
        const int ci = (ty + 2) * SM::CW + tx + 2;
        const int mi = (ty + 1) * SM::MW + tx + 1;
        const long hi = long(gy - ya) * g.nx + gx;
        if (sm.m[ci]) {
            for (int f = 0; f < 10; ++f) out[f * n + hi] = 0.0;
            continue;
        }
        const Nb nb = make_nb(g, gx, gy);
        R gg[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) gg[k] = ld<P>(src, c, 18 + k, g.npad, nb.up(k));
        NodeMacro<R> o = node_macro<R>(tile_stencil<P, TY>(sm, ci, mi), c, gg);
        out[0 * n + hi] = double(o.c1);
        out[1 * n + hi] = double(o.c2);
        out[2 * n + hi] = double(R(1) - o.c1 - o.c2);
        out[3 * n + hi] = double(o.rho);
        out[4 * n + hi] = double(o.ux);
        out[5 * n + hi] = double(o.uy);
        out[6 * n + hi] = double(o.p);
        out[7 * n + hi] = double(o.mu1);
        out[8 * n + hi] = double(o.mu2);
        out[9 * n + hi] = double(sm.mu3[mi]);
    }
}

// ------------------------------------------------------------ populations
// f(x) of the rows [ya, yb) as doubles, [27][(yb - ya) * nx]
template <int P>
__global__ __launch_bounds__(kThreads) void populations_kernel(Grid g, Consts<typename Tr<P>::R> c,
                                                               const uint8_t* __restrict__ mat,
                                                               PopBuf src, int ya, int yb,
                                                               double* __restrict__ out) {
    const long n = long(g.nx) * (yb - ya);
    for (long hi = long(blockIdx.x) * kThreads + threadIdx.x; hi < n;
         hi += long(gridDim.x) * kThreads) {
        const int by = int(hi / g.nx), gx = int(hi - long(by) * g.nx);
        const int gy = ya + by;
        const Nb nb = make_nb(g, gx, gy);
        const bool solid = mat[nb.r0 + gx] != 0;
#pragma unroll
        for (int q = 0; q < 27; ++q)
            out[q * n + hi] = solid ? 0.0 : double(ld<P>(src, c, q, g.npad, nb.up(q % 9)));
    }
}

// ------------------------------------------------------------------- mass
// Per-component mass and health check (row a7 of the path).  The sums
// sum_x c_i over the fluid nodes are conserved by the step (the equilibria
// and sources of Eqs. 2a and 11a carry no mass, Eq. 3 fixes c3, half-way
// bounce-back of Eq. 44 returns every population), so they are read from the
// history planes (c1, c2, ux, uy of the state the last step started from,
// which holds the same sums as the current populations up to rounding): 16
// or 32 bytes per node instead of 18 pulled populations.  A node whose c1,
// c2, ux or uy is not finite is counted (u carries the g moments).
// Deterministic: block b owns a fixed contiguous range of the padded node
// index space; each thread sums its nodes in order, each wavefront reduces
// with a fixed butterfly of lane exchanges, and the four wavefronts' sums are
// added in wave order; one block then reduces the per-block partials the same
// way.

// the four sums of a wavefront, in every lane (fixed exchange pattern)
__device__ __forceinline__ void wave_sum4(double (&v)[4]) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], m, 64);
}

// block-wide sums of v (kThreads threads, four wavefronts) into out[0..3]
__device__ __forceinline__ void block_sum4(double (&v)[4], double* out) {
    __shared__ double wsum[kThreads / 64][4];
    wave_sum4(v);
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) wsum[wv][q] = v[q];
    __syncthreads();
    if (threadIdx.x < 4) {
        double a = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) a += wsum[w][threadIdx.x];
        out[threadIdx.x] = a;
    }
}

template <typename H>
__global__ __launch_bounds__(kThreads) void mass_partial_kernel(Grid g,
                                                                const uint8_t* __restrict__ mat,
                                                                const H* __restrict__ hist,
                                                                double* __restrict__ part) {
    const long n = g.npad;
    const long per = (n + gridDim.x - 1) / gridDim.x;
    const long lo = long(blockIdx.x) * per;
    const long end = lo + per < n ? lo + per : n;
    double v[4] = {0.0, 0.0, 0.0, 0.0};    // sum c1, sum c2, sum c3, non-finite count
    for (long i = lo + threadIdx.x; i < end; i += kThreads) {
        const int x = int(i % g.pitch);
        if (x >= g.nx || mat[i]) continue;
        const double a = double(hist[i]), b = double(hist[n + i]);
        const double ux = double(hist[2 * n + i]), uy = double(hist[3 * n + i]);
        if (!isfinite(a) || !isfinite(b) || !isfinite(ux) || !isfinite(uy)) v[3] += 1.0;
        v[0] += a;
        v[1] += b;
        v[2] += 1.0 - a - b;
    }
    block_sum4(v, part + 4 * blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void mass_final_kernel(const double* __restrict__ part,
                                                              int nparts, double* __restrict__ out) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kThreads)
        for (int q = 0; q < 4; ++q) v[q] += part[4 * i + q];
    block_sum4(v, out);
}

template <int P>
using CT = Consts<typename Tr<P>::R>;

template <int P, unsigned F>
void step_pf(const void* descs, int ndesc, int total_tiles, int parity, hipStream_t s) {
    hipLaunchKernelGGL((step_kernel<P, F>), dim3(total_tiles), dim3(kStepThreads), 0, s,
                       static_cast<const unsigned char*>(descs), ndesc, total_tiles, parity);
}

template <int P, unsigned F>
void step2_p(const void* descs, int ndesc, int total_tiles, int parity, hipStream_t s) {
    hipLaunchKernelGGL((step2_kernel<P, F>), dim3(total_tiles), dim3(kStep2Threads), 0, s,
                       static_cast<const unsigned char*>(descs), ndesc, total_tiles, parity);
}

template <int P>
hipError_t step_p(unsigned features, const void* descs, int ndesc, int total_tiles, int parity,
                  hipStream_t s) {
    switch (features & (kFeatVel | kFeatLam)) {
        case 0: step_pf<P, 0>(descs, ndesc, total_tiles, parity, s); break;
        case kFeatVel: step_pf<P, kFeatVel>(descs, ndesc, total_tiles, parity, s); break;
        case kFeatLam: step_pf<P, kFeatLam>(descs, ndesc, total_tiles, parity, s); break;
        default: step_pf<P, kFeatVel | kFeatLam>(descs, ndesc, total_tiles, parity, s); break;
    }
    return hipGetLastError();
}

constexpr int kAuxRows = 8;  // tile rows of the init / readout kernels

}  // namespace

hipError_t launch_step(int prec, unsigned features, const void* descs, int ndesc,
                       int total_tiles, int parity, hipStream_t s) {
    switch (prec) {
        case P64: return step_p<P64>(features, descs, ndesc, total_tiles, parity, s);
        case P32: return step_p<P32>(features, descs, ndesc, total_tiles, parity, s);
        case P16: return step_p<P16>(features, descs, ndesc, total_tiles, parity, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2(int prec, unsigned features, const void* descs, int ndesc,
                        int total_tiles, int parity, hipStream_t s) {
    if (prec != P32) return hipErrorInvalidValue;
    switch (features & (kFeatVel | kFeatLam)) {
        case 0: step2_p<P32, 0>(descs, ndesc, total_tiles, parity, s); break;
        case kFeatVel: step2_p<P32, kFeatVel>(descs, ndesc, total_tiles, parity, s); break;
        case kFeatLam: step2_p<P32, kFeatLam>(descs, ndesc, total_tiles, parity, s); break;
        default: step2_p<P32, kFeatVel | kFeatLam>(descs, ndesc, total_tiles, parity, s); break;
    }
    return hipGetLastError();
}

template <int P>
static hipError_t init_p(const Grid& g, const void* consts, const uint8_t* mat,
                         const double* mtab, const double* in4, PopBuf dst, void* hist,
                         hipStream_t s) {
    int nt = ((g.nx + kTileX - 1) / kTileX) * ((g.ny + kAuxRows - 1) / kAuxRows);
    hipLaunchKernelGGL((init_kernel<P, kAuxRows>), dim3(nt), dim3(kThreads), 0, s, g,
                       *static_cast<const CT<P>*>(consts), mat, mtab, in4, dst,
                       static_cast<typename Tr<P>::H*>(hist));
    return hipGetLastError();
}

hipError_t launch_init(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                       const double* mtab, const double* in4, PopBuf dst, void* hist,
                       hipStream_t s) {
    switch (prec) {
        case P64: return init_p<P64>(g, consts, mat, mtab, in4, dst, hist, s);
        case P32: return init_p<P32>(g, consts, mat, mtab, in4, dst, hist, s);
        case P16: return init_p<P16>(g, consts, mat, mtab, in4, dst, hist, s);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t readout_p(const Grid& g, const void* consts, const uint8_t* mat,
                            const double* mtab, PopBuf src, int ya, int yb, double* out,
                            hipStream_t s) {
    int nt = ((g.nx + kTileX - 1) / kTileX) * ((yb - ya + kAuxRows - 1) / kAuxRows);
    hipLaunchKernelGGL((readout_kernel<P, kAuxRows>), dim3(nt), dim3(kThreads), 0, s, g,
                       *static_cast<const CT<P>*>(consts), mat, mtab, src, ya, yb, out);
    return hipGetLastError();
}

hipError_t launch_readout(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                          const double* mtab, PopBuf src, int ya, int yb, double* out10,
                          hipStream_t s) {
    if (ya < 0 || yb > g.ny || ya >= yb) return hipErrorInvalidValue;
    switch (prec) {
        case P64: return readout_p<P64>(g, consts, mat, mtab, src, ya, yb, out10, s);
        case P32: return readout_p<P32>(g, consts, mat, mtab, src, ya, yb, out10, s);
        case P16: return readout_p<P16>(g, consts, mat, mtab, src, ya, yb, out10, s);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t pops_p(const Grid& g, const void* consts, const uint8_t* mat, PopBuf src,
                         int ya, int yb, double* out, hipStream_t s) {
    long n = long(g.nx) * (yb - ya);
    int nb = int((n + kThreads - 1) / kThreads);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL((populations_kernel<P>), dim3(nb), dim3(kThreads), 0, s, g,
                       *static_cast<const CT<P>*>(consts), mat, src, ya, yb, out);
    return hipGetLastError();
}

hipError_t launch_populations(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                              PopBuf src, int ya, int yb, double* out27, hipStream_t s) {
    if (ya < 0 || yb > g.ny || ya >= yb) return hipErrorInvalidValue;
    switch (prec) {
        case P64: return pops_p<P64>(g, consts, mat, src, ya, yb, out27, s);
        case P32: return pops_p<P32>(g, consts, mat, src, ya, yb, out27, s);
        case P16: return pops_p<P16>(g, consts, mat, src, ya, yb, out27, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename H>
static hipError_t mass_h(const Grid& g, const uint8_t* mat, const void* hist, double* part,
                         double* result, hipStream_t s) {
    hipLaunchKernelGGL((mass_partial_kernel<H>), dim3(kReduceBlocks), dim3(kThreads), 0, s, g,
                       mat, static_cast<const H*>(hist), part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mass_final_kernel, dim3(1), dim3(kThreads), 0, s, part, kReduceBlocks,
                       result);
    return hipGetLastError();
}

hipError_t mass_scratch(double** out) {
    static std::mutex mu;
    static double* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // resolved once per device, with that device current: each GPU holds
        // its own copy of the array at its own address
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_mass(int prec, const Grid& g, const uint8_t* mat, const void* hist,
                       double* partials, double* result, hipStream_t s) {
    switch (prec) {
        case P64: return mass_h<double>(g, mat, hist, partials, result, s);
        case P32:
        case P16: return mass_h<float>(g, mat, hist, partials, result, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tlb
