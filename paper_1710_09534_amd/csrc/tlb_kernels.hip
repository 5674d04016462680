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
// One step is one kernel.  A workgroup owns a 64 x TY tile and
//   A. pulls f^1, f^2 on the tile plus a 2-node halo and forms c1, c2 in LDS
//      (Eqs. 3, 13a),
//   B. forms the chemical potentials on the tile plus a 1-node halo with the
//      wetting ghosts of Eq. 42 across solid links (Eqs. 8, 20b),
//   C. per interior node: gradients with the symmetric ghost rule (Eq. 43),
//      surface-tension force, velocity, interfacial force, pressure,
//      Euler time derivative, equilibria, sources and BGK collision
//      (Eqs. 2, 4, 11-15, 18b, 19, 45), and the coalesced stores.
// Workgroup ids are remapped so that each of the eight XCDs walks one
// contiguous band of tiles: halo re-reads then hit that XCD's L2.
#include <hip/hip_runtime.h>

#include "tlb_internal.h"

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

template <int P>
__device__ __forceinline__ typename Tr<P>::R ld(const PopBuf& b, const Consts<typename Tr<P>::R>& c,
                                                int q, long npad, long i) {
    if constexpr (P == P16) {
        if (q == 0 || q == 9) return b.rest[(q / 9) * npad + i];
        return float(static_cast<const _Float16*>(b.planes)[q * npad + i]) * c.iscale[q / 9];
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
        } else {
            static_cast<_Float16*>(b.planes)[q * npad + i] = _Float16(v * c.scale[q / 9]);
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

// Phase B: chemical potentials (Eq. 8) on the mu region; the Laplacian of
// c_i (Eq. 20b) sees, across a link into a solid node of material m, the
// ghost c_i + (4/D) h_i(c) of Eq. 42 evaluated at the fluid node itself.
template <int P, int TY>
__device__ __forceinline__ void phase_b(Smem<P, TY>& sm, const Consts<typename Tr<P>::R>& c) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    for (int i = threadIdx.x; i < SM::MH * SM::MW; i += kThreads) {
        int my = i / SM::MW;
        int mx = i - my * SM::MW;
        int ci = (my + 1) * SM::CW + mx + 1;
        R mu1 = R(0), mu2 = R(0), mu3 = R(0);
        if (sm.m[ci] == 0) {
            R c1 = sm.c1[ci], c2 = sm.c2[ci];
            R c3 = R(1) - c1 - c2;
            R l1 = R(0), l2 = R(0), l3 = R(0);
#pragma unroll
            for (int k = 1; k < 9; ++k) {
                int ni = ci + EY[k] * SM::CW + EX[k];
                int mn = sm.m[ni];
                R n1, n2, n3;
                if (mn) {
                    const R* t = &sm.mt[kMatStride * mn];
                    R h1 = t[1] * c1 * c3 + t[0] * c1 * c2;
                    R h2 = -t[0] * c1 * c2 + t[2] * c2 * c3;
                    R h3 = -t[2] * c2 * c3 - t[1] * c1 * c3;
                    n1 = c1 + c.k4D * h1;
                    n2 = c2 + c.k4D * h2;
                    n3 = c3 + c.k4D * h3;
                } else {
                    n1 = sm.c1[ni];
                    n2 = sm.c2[ni];
                    n3 = R(1) - n1 - n2;
                }
                l1 += wgt<R>(k) * (n1 - c1);
                l2 += wgt<R>(k) * (n2 - c2);
                l3 += wgt<R>(k) * (n3 - c3);
            }
            l1 *= R(6);  // 2 / c_s^2
            l2 *= R(6);
            l3 *= R(6);
            R tri = R(2) * c.lamT * c1 * c2 * (R(1) - c1 - c2);
            mu1 = c.k12D * (c.lam1 * c1 * (R(1) - c1) * (R(1) - R(2) * c1) - tri) - c.k34D * c.lam1 * l1;
            mu2 = c.k12D * (c.lam2 * c2 * (R(1) - c2) * (R(1) - R(2) * c2) - tri) - c.k34D * c.lam2 * l2;
            mu3 = c.k12D * (c.lam3 * c3 * (R(1) - c3) * (R(1) - R(2) * c3) - tri) - c.k34D * c.lam3 * l3;
        }
        sm.mu1[i] = mu1;
        sm.mu2[i] = mu2;
        sm.mu3[i] = mu3;
    }
}

// Macroscopic state of one interior node (phase C front half).
template <typename R>
struct NodeMacro {
    R c1, c2, rho, itg, mu1, mu2, ux, uy, p, grx, gry, fx, fy, fax, fay;
};

// Gradients (Eq. 20a, symmetric ghosts of Eq. 43), forces, velocity
// (Eq. 13b), interfacial force (Eq. 12) and pressure (Eq. 13c) from the
// pulled g and the LDS fields.
template <int P, int TY>
__device__ __forceinline__ NodeMacro<typename Tr<P>::R> node_macro(
    const Smem<P, TY>& sm, const Consts<typename Tr<P>::R>& c, int ci, int mi,
    const typename Tr<P>::R* gg) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    NodeMacro<R> o;
    R c1 = sm.c1[ci], c2 = sm.c2[ci];
    R mu1 = sm.mu1[mi], mu2 = sm.mu2[mi], mu3 = sm.mu3[mi];
    R g1x = R(0), g1y = R(0), g2x = R(0), g2y = R(0), lm1 = R(0), lm2 = R(0);
#pragma unroll
    for (int k = 1; k < 9; ++k) {
        int ni = ci + EY[k] * SM::CW + EX[k];
        int nmi = mi + EY[k] * SM::MW + EX[k];
        bool solid = sm.m[ni] != 0;
        R v1 = solid ? c1 : sm.c1[ni];
        R v2 = solid ? c2 : sm.c2[ni];
        R w1 = solid ? mu1 : sm.mu1[nmi];
        R w2 = solid ? mu2 : sm.mu2[nmi];
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
    R g3x = -(g1x + g2x), g3y = -(g1y + g2y);              // c3 = 1 - c1 - c2
    R rho = c.rho3 + c.drho1 * c1 + c.drho2 * c2;          // Eq. 14
    R nu = c.nu3 + c.dnu1 * c1 + c.dnu2 * c2;              // Eq. 15
    R taug = R(3) * nu + R(0.5);                           // Eq. 18b
    R grx = c.drho1 * g1x + c.drho2 * g2x;                 // grad rho
    R gry = c.drho1 * g1y + c.drho2 * g2y;
    R fsx = mu1 * g1x + mu2 * g2x + mu3 * g3x;             // F_s
    R fsy = mu1 * g1y + mu2 * g2y + mu3 * g3y;
    R fx = fsx + rho * c.gx;
    R fy = fsy + rho * c.gy;
    R mx = R(0), my = R(0), sum = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        if (EX[k]) mx += R(EX[k]) * gg[k];
        if (EY[k]) my += R(EY[k]) * gg[k];
        if (k) sum += gg[k];
    }
    R irho = R(1) / rho;
    R ux = (mx + R(0.5) * fx) * irho;
    R uy = (my + R(0.5) * fy) * irho;
    R a = c.am1 * lm1 + c.am2 * lm2;
    R uu = ux * ux + uy * uy;
    // c_s^2/(1-w0) = 3/5; s_0(u) = -w0 u.u/(2 c_s^2) = -(2/3) u.u
    R p = R(0.6) * (sum + R(0.5) * (ux * grx + uy * gry) - rho * (R(2) / R(3)) * uu);
    o.c1 = c1; o.c2 = c2; o.rho = rho; o.itg = R(1) / taug;
    o.mu1 = mu1; o.mu2 = mu2; o.ux = ux; o.uy = uy; o.p = p;
    o.grx = grx; o.gry = gry; o.fx = fx; o.fy = fy; o.fax = ux * a; o.fay = uy * a;
    return o;
}

// ------------------------------------------------------------------- step
template <int P, int TY>
__global__ __launch_bounds__(kThreads) void step_kernel(Grid g, Consts<typename Tr<P>::R> c,
                                                        const uint8_t* __restrict__ mat,
                                                        const double* __restrict__ mtab,
                                                        PopBuf src, PopBuf dst,
                                                        typename Tr<P>::H* __restrict__ hist) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    __shared__ SM sm;
    const int t = tile_of(blockIdx.x, g.tiles_x * g.tiles_y);
    const int x0 = (t % g.tiles_x) * kTileX;
    const int y0 = (t / g.tiles_x) * TY;
    load_mtab<P, TY>(sm, mtab);
    phase_a<P, TY, true>(sm, g, c, mat, src, nullptr, x0, y0);
    __syncthreads();
    phase_b<P, TY>(sm, c);
    __syncthreads();

    const int tx = threadIdx.x & (kTileX - 1);
    const int gx = x0 + tx;
    if (gx >= g.nx) return;
    for (int ty = threadIdx.x / kTileX; ty < TY; ty += kThreads / kTileX) {
        const int gy = y0 + ty;
        if (gy >= g.ny) break;
        const int ci = (ty + 2) * SM::CW + tx + 2;
        const int mi = (ty + 1) * SM::MW + tx + 1;
        if (sm.m[ci]) continue;
        const Nb nb = make_nb(g, gx, gy);
        const long idx = nb.r0 + gx;
        R f1[9], f2[9], gg[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            long j = nb.up(k);
            f1[k] = ld<P>(src, c, k, g.npad, j);
            f2[k] = ld<P>(src, c, 9 + k, g.npad, j);
            gg[k] = ld<P>(src, c, 18 + k, g.npad, j);
        }
        const R c1o = R(hist[idx]), c2o = R(hist[g.npad + idx]);
        const R uxo = R(hist[2 * g.npad + idx]), uyo = R(hist[3 * g.npad + idx]);
        NodeMacro<R> o = node_macro<P, TY>(sm, c, ci, mi, gg);
        // Euler time derivative of c_i u (Eq. 19 inside Eq. 11a)
        const R d1x = o.c1 * o.ux - c1o * uxo, d1y = o.c1 * o.uy - c1o * uyo;
        const R d2x = o.c2 * o.ux - c2o * uxo, d2y = o.c2 * o.uy - c2o * uyo;
        hist[idx] = typename Tr<P>::H(o.c1);
        hist[g.npad + idx] = typename Tr<P>::H(o.c2);
        hist[2 * g.npad + idx] = typename Tr<P>::H(o.ux);
        hist[3 * g.npad + idx] = typename Tr<P>::H(o.uy);

        const R uu = o.ux * o.ux + o.uy * o.uy;
        const R em1 = c.eta1 * o.mu1, em2 = c.eta2 * o.mu2;
        const R p3 = R(3) * o.p;
        const R fsg = R(1) - R(0.5) * o.itg;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const R w = wgt<R>(k);
            const R eu = R(EX[k]) * o.ux + R(EY[k]) * o.uy;
            // Eq. 2a
            R fe1, fe2, ge;
            const R sk = w * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);  // Eq. 4
            if (k == 0) {
                fe1 = o.c1 + (w - R(1)) * em1;
                fe2 = o.c2 + (w - R(1)) * em2;
                ge = p3 * (w - R(1)) + o.rho * sk;                           // Eq. 2b
            } else {
                fe1 = w * (em1 + R(3) * o.c1 * eu);
                fe2 = w * (em2 + R(3) * o.c2 * eu);
                ge = p3 * w + o.rho * sk;
            }
            // Eq. 11a, Eq. 11b
            const R ed1 = R(EX[k]) * d1x + R(EY[k]) * d1y;
            const R ed2 = R(EX[k]) * d2x + R(EY[k]) * d2y;
            const R bx = sk * o.grx + (sk + w) * R(3) * o.fx;
            const R by = sk * o.gry + (sk + w) * R(3) * o.fy;
            const R gk = fsg * ((R(EX[k]) - o.ux) * bx + (R(EY[k]) - o.uy) * by)
                       + R(3) * w * (R(EX[k]) * o.fax + R(EY[k]) * o.fay);
            // BGK collision (Eq. 45)
            f1[k] = f1[k] + (fe1 - f1[k]) * c.itau1 + c.fs1 * R(3) * w * ed1;
            f2[k] = f2[k] + (fe2 - f2[k]) * c.itau2 + c.fs2 * R(3) * w * ed2;
            gg[k] = gg[k] + (ge - gg[k]) * o.itg + gk;
            st<P>(dst, c, k, g.npad, idx, f1[k]);
            st<P>(dst, c, 9 + k, g.npad, idx, f2[k]);
            st<P>(dst, c, 18 + k, g.npad, idx, gg[k]);
        }
        // half-way bounce-back into solid neighbours (Eq. 44), with the
        // moving-wall term -2 w_k a e_k.u_w / c_s^2 (a = c_i for f^i, rho for g)
#pragma unroll
        for (int k = 1; k < 9; ++k) {
            const int mn = sm.m[ci + EY[k] * SM::CW + EX[k]];
            if (mn) {
                const R* tm = &sm.mt[kMatStride * mn];
                const R corr = -R(6) * wgt<R>(k) * (R(EX[k]) * tm[3] + R(EY[k]) * tm[4]);
                const long s = nb.dn(k);
                st<P>(dst, c, OPP[k], g.npad, s, f1[k] + corr * o.c1);
                st<P>(dst, c, 9 + OPP[k], g.npad, s, f2[k] + corr * o.c2);
                st<P>(dst, c, 18 + OPP[k], g.npad, s, gg[k] + corr * o.rho);
            }
        }
    }
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
    const int x0 = (t % g.tiles_x) * kTileX;
    const int y0 = (t / g.tiles_x) * TY;
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
                                                           PopBuf src, double* __restrict__ out) {
    using R = typename Tr<P>::R;
    using SM = Smem<P, TY>;
    __shared__ SM sm;
    const int t = blockIdx.x;
    const int x0 = (t % g.tiles_x) * kTileX;
    const int y0 = (t / g.tiles_x) * TY;
    load_mtab<P, TY>(sm, mtab);
    phase_a<P, TY, true>(sm, g, c, mat, src, nullptr, x0, y0);
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
        const long hi = long(gy) * g.nx + gx;
        if (sm.m[ci]) {
            for (int f = 0; f < 10; ++f) out[f * n + hi] = 0.0;
            continue;
        }
        const Nb nb = make_nb(g, gx, gy);
        R gg[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) gg[k] = ld<P>(src, c, 18 + k, g.npad, nb.up(k));
        NodeMacro<R> o = node_macro<P, TY>(sm, c, ci, mi, gg);
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
template <int P>
__global__ __launch_bounds__(kThreads) void populations_kernel(Grid g, Consts<typename Tr<P>::R> c,
                                                               const uint8_t* __restrict__ mat,
                                                               PopBuf src, double* __restrict__ out) {
    const long n = long(g.nx) * g.ny;
    for (long hi = long(blockIdx.x) * kThreads + threadIdx.x; hi < n;
         hi += long(gridDim.x) * kThreads) {
        const int gy = int(hi / g.nx), gx = int(hi - long(gy) * g.nx);
        const Nb nb = make_nb(g, gx, gy);
        const bool solid = mat[nb.r0 + gx] != 0;
#pragma unroll
        for (int q = 0; q < 27; ++q)
            out[q * n + hi] = solid ? 0.0 : double(ld<P>(src, c, q, g.npad, nb.up(q % 9)));
    }
}

// ------------------------------------------------------------------- mass
// Deterministic two-pass reduction: block b sums a fixed contiguous range
// of nodes with a fixed tree; one block then sums the partials.
template <int P>
__global__ __launch_bounds__(kThreads) void mass_partial_kernel(Grid g, Consts<typename Tr<P>::R> c,
                                                                const uint8_t* __restrict__ mat,
                                                                PopBuf src, double* __restrict__ part) {
    __shared__ double red[4][kThreads];
    const long n = long(g.nx) * g.ny;
    const long per = (n + gridDim.x - 1) / gridDim.x;
    const long lo = long(blockIdx.x) * per;
    const long hi_end = lo + per < n ? lo + per : n;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, bad = 0.0;
    for (long hi = lo + threadIdx.x; hi < hi_end; hi += kThreads) {
        const int gy = int(hi / g.nx), gx = int(hi - long(gy) * g.nx);
        const Nb nb = make_nb(g, gx, gy);
        if (mat[nb.r0 + gx]) continue;
        typename Tr<P>::R a = 0, b = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            long j = nb.up(k);
            a += ld<P>(src, c, k, g.npad, j);
            b += ld<P>(src, c, 9 + k, g.npad, j);
        }
        const double da = double(a), db = double(b);
        if (!isfinite(da) || !isfinite(db)) bad += 1.0;
        s1 += da;
        s2 += db;
        s3 += 1.0 - da - db;
    }
    red[0][threadIdx.x] = s1;
    red[1][threadIdx.x] = s2;
    red[2][threadIdx.x] = s3;
    red[3][threadIdx.x] = bad;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kThreads) void mass_final_kernel(const double* __restrict__ part,
                                                              int nparts, double* __restrict__ out) {
    __shared__ double red[4][kThreads];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kThreads)
        for (int q = 0; q < 4; ++q) s[q] += part[i * 4 + q];
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

template <int P>
using CT = Consts<typename Tr<P>::R>;

template <int P, int TY>
hipError_t step_ty(const Grid& g, const void* consts, const uint8_t* mat, const double* mtab,
                   PopBuf src, PopBuf dst, void* hist, hipStream_t s) {
    int nt = g.tiles_x * g.tiles_y;
    hipLaunchKernelGGL((step_kernel<P, TY>), dim3(nt), dim3(kThreads), 0, s, g,
                       *static_cast<const CT<P>*>(consts), mat, mtab, src, dst,
                       static_cast<typename Tr<P>::H*>(hist));
    return hipGetLastError();
}

template <int P>
hipError_t step_p(const Grid& g, const void* consts, const uint8_t* mat, const double* mtab,
                  PopBuf src, PopBuf dst, void* hist, hipStream_t s) {
    switch (g.tile_rows) {
        case 2: return step_ty<P, 2>(g, consts, mat, mtab, src, dst, hist, s);
        case 4: return step_ty<P, 4>(g, consts, mat, mtab, src, dst, hist, s);
        case 8: return step_ty<P, 8>(g, consts, mat, mtab, src, dst, hist, s);
        case 16: return step_ty<P, 16>(g, consts, mat, mtab, src, dst, hist, s);
        default: return hipErrorInvalidValue;
    }
}

constexpr int kAuxRows = 8;  // tile rows of the init / readout kernels

}  // namespace

hipError_t launch_step(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                       const double* mtab, PopBuf src, PopBuf dst, void* hist,
                       hipStream_t s) {
    switch (prec) {
        case P64: return step_p<P64>(g, consts, mat, mtab, src, dst, hist, s);
        case P32: return step_p<P32>(g, consts, mat, mtab, src, dst, hist, s);
        case P16: return step_p<P16>(g, consts, mat, mtab, src, dst, hist, s);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t init_p(const Grid& g, const void* consts, const uint8_t* mat,
                         const double* mtab, const double* in4, PopBuf dst, void* hist,
                         hipStream_t s) {
    int nt = g.tiles_x * ((g.ny + kAuxRows - 1) / kAuxRows);
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
                            const double* mtab, PopBuf src, double* out, hipStream_t s) {
    int nt = g.tiles_x * ((g.ny + kAuxRows - 1) / kAuxRows);
    hipLaunchKernelGGL((readout_kernel<P, kAuxRows>), dim3(nt), dim3(kThreads), 0, s, g,
                       *static_cast<const CT<P>*>(consts), mat, mtab, src, out);
    return hipGetLastError();
}

hipError_t launch_readout(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                          const double* mtab, PopBuf src, void* /*hist*/, double* out10,
                          hipStream_t s) {
    switch (prec) {
        case P64: return readout_p<P64>(g, consts, mat, mtab, src, out10, s);
        case P32: return readout_p<P32>(g, consts, mat, mtab, src, out10, s);
        case P16: return readout_p<P16>(g, consts, mat, mtab, src, out10, s);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t pops_p(const Grid& g, const void* consts, const uint8_t* mat, PopBuf src,
                         double* out, hipStream_t s) {
    long n = long(g.nx) * g.ny;
    int nb = int((n + kThreads - 1) / kThreads);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL((populations_kernel<P>), dim3(nb), dim3(kThreads), 0, s, g,
                       *static_cast<const CT<P>*>(consts), mat, src, out);
    return hipGetLastError();
}

hipError_t launch_populations(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                              PopBuf src, double* out27, hipStream_t s) {
    switch (prec) {
        case P64: return pops_p<P64>(g, consts, mat, src, out27, s);
        case P32: return pops_p<P32>(g, consts, mat, src, out27, s);
        case P16: return pops_p<P16>(g, consts, mat, src, out27, s);
        default: return hipErrorInvalidValue;
    }
}

template <int P>
static hipError_t mass_p(const Grid& g, const void* consts, const uint8_t* mat, PopBuf src,
                         double* part, double* result, hipStream_t s) {
    hipLaunchKernelGGL((mass_partial_kernel<P>), dim3(kReduceBlocks), dim3(kThreads), 0, s, g,
                       *static_cast<const CT<P>*>(consts), mat, src, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mass_final_kernel, dim3(1), dim3(kThreads), 0, s, part, kReduceBlocks,
                       result);
    return hipGetLastError();
}

hipError_t launch_mass(int prec, const Grid& g, const void* consts, const uint8_t* mat,
                       PopBuf src, double* partials, double* result, hipStream_t s) {
    switch (prec) {
        case P64: return mass_p<P64>(g, consts, mat, src, partials, result, s);
        case P32: return mass_p<P32>(g, consts, mat, src, partials, result, s);
        case P16: return mass_p<P16>(g, consts, mat, src, partials, result, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tlb
