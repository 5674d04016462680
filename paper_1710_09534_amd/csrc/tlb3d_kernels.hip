// tlb3d_kernels.hip -- gfx950 kernels of the three-dimensional (D3Q19)
// version of the ternary wetting lattice Boltzmann step (Liang et al.,
// arXiv:1710.09534; the model is stated on D2Q9 "without loss of
// generality", Sec. II.A, and carried to D3Q19 link by link).
//
// One step is three launches over a grid of 64 x 4 node blocks per z-plane:
//   c3_kernel   pulls f^1, f^2 (38 planes) and stores c1, c2 (Eqs. 3, 13a);
//   mu3_kernel  forms the chemical potentials from c with the wetting ghosts
//               of Eq. 42 across wall links (Eqs. 8, 20b; Eq. 6 for
//               lambda > 0) and stores mu1, mu2, mu3;
//   col3_kernel pulls all 57 populations, forms gradients with the symmetric
//               ghosts of Eq. 43, forces, velocity, interfacial force,
//               pressure and the Euler time derivative (Eqs. 12-15, 18b, 19),
//               collides (Eqs. 2, 4, 11, 45) and stores the 57 post-collision
//               populations, with half-way bounce-back (Eq. 44) folded into
//               the stores: a fluid node whose neighbour x + e_k is a wall
//               writes f'_k(x) (plus the moving-wall term) into slot
//               P_opp(k) of that wall node, the slot only x pulls from.
// Three-dimensional stencils need a radius-2 halo of c in every direction,
// which a fused kernel would recompute for a large fraction of each tile;
// splitting at c and mu costs 2 + 3 values per node instead.
#include <hip/hip_runtime.h>

#include "tlb3d_internal.h"

namespace tlb3 {
namespace {

// D3Q19: k = 0 rest; 1-6 axis links (+x, -x, +y, -y, +z, -z); 7-18 edge
// diagonals in pairs (e, -e).
constexpr int EX[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }

template <typename R>
__device__ __forceinline__ constexpr R wq(int k) {
    return k == 0 ? R(1) / R(3) : (k < 7 ? R(1) / R(18) : R(1) / R(36));
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Wrapped neighbourhood of (x, y, z): row bases for y-1..y+1, z-1..z+1 and
// columns x-1..x+1.
struct Nb3 {
    long long row[3][3];
    int xs[3];
    __device__ __forceinline__ long long at(int dx, int dy, int dz) const {
        return row[dy + 1][dz + 1] + xs[dx + 1];
    }
};

__device__ __forceinline__ Nb3 make_nb3(const Grid3& g, int x, int y, int z) {
    Nb3 n;
    const int ys[3] = {wrap(y - 1, g.ny), y, wrap(y + 1, g.ny)};
    const int zs[3] = {wrap(z - 1, g.nz), z, wrap(z + 1, g.nz)};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            n.row[a][b] = ((long long)zs[b] * g.ny + ys[a]) * g.pitch;
    n.xs[0] = wrap(x - 1, g.nx);
    n.xs[1] = x;
    n.xs[2] = wrap(x + 1, g.nx);
    return n;
}

struct Node {
    int x, y, z;
    bool in;
};

__device__ __forceinline__ Node node_of(const Grid3& g) {
    Node p;
    p.x = blockIdx.x * kBlockX + int(threadIdx.x % kBlockX);
    p.y = blockIdx.y * kBlockY + int(threadIdx.x / kBlockX);
    p.z = blockIdx.z;
    p.in = p.x < g.nx && p.y < g.ny;
    return p;
}

// ------------------------------------------------------------ order parameters
template <typename R>
__global__ __launch_bounds__(256) void c3_kernel(Grid3 g, Bufs3<R> b, int cur) {
    const Node p = node_of(g);
    if (!p.in) return;
    const Nb3 nb = make_nb3(g, p.x, p.y, p.z);
    const long long i = nb.at(0, 0, 0);
    const R* __restrict__ P = b.pop[cur];
    R a = R(0), c = R(0);
    if (!b.mat[i]) {
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            const long long j = nb.at(-EX[k], -EY[k], -EZ[k]);
            a += P[k * g.npad + j];
            c += P[(kQ + k) * g.npad + j];
        }
    }
    b.cf[i] = a;
    b.cf[g.npad + i] = c;
}

// --------------------------------------------------------- chemical potentials
template <typename R>
__global__ __launch_bounds__(256) void mu3_kernel(Grid3 g, Consts3<R> c, Bufs3<R> b) {
    const Node p = node_of(g);
    if (!p.in) return;
    const Nb3 nb = make_nb3(g, p.x, p.y, p.z);
    const long long i = nb.at(0, 0, 0);
    R mu1 = R(0), mu2 = R(0), mu3 = R(0);
    if (!b.mat[i]) {
        const R c1 = b.cf[i], c2 = b.cf[g.npad + i], c3 = R(1) - c1 - c2;
        R l1 = R(0), l2 = R(0), l3 = R(0);
#pragma unroll
        for (int k = 1; k < kQ; ++k) {
            const long long j = nb.at(EX[k], EY[k], EZ[k]);
            const int m = b.mat[j];
            R n1, n2, n3;
            if (m) {
                // Eq. 42: ghost seen across a wall link, wall value c(x)
                const double* t = &b.mtab[kMatStride * m];
                const R c12 = R(t[0]), c13 = R(t[1]), c23 = R(t[2]);
                n1 = c1 + c.k4D * (c13 * c1 * c3 + c12 * c1 * c2);
                n2 = c2 + c.k4D * (-c12 * c1 * c2 + c23 * c2 * c3);
                n3 = c3 + c.k4D * (-c23 * c2 * c3 - c13 * c1 * c3);
            } else {
                n1 = b.cf[j];
                n2 = b.cf[g.npad + j];
                n3 = R(1) - n1 - n2;
            }
            l1 += wq<R>(k) * (n1 - c1);
            l2 += wq<R>(k) * (n2 - c2);
            l3 += wq<R>(k) * (n3 - c3);
        }
        l1 *= R(6);
        l2 *= R(6);
        l3 *= R(6);
        const R tri = R(2) * c.lamT * c1 * c2 * c3;
        mu1 = c.k12D * (c.lam1 * c1 * (R(1) - c1) * (R(1) - R(2) * c1) - tri) - c.k34D * c.lam1 * l1;
        mu2 = c.k12D * (c.lam2 * c2 * (R(1) - c2) * (R(1) - R(2) * c2) - tri) - c.k34D * c.lam2 * l2;
        mu3 = c.k12D * (c.lam3 * c3 * (R(1) - c3) * (R(1) - R(2) * c3) - tri) - c.k34D * c.lam3 * l3;
        if (c.kB != R(0)) {
            // lambda c1^2 c2^2 c3^2 term of Eq. 5 through Eq. 6
            const R t = c.kB * c1 * c2 * c3;
            mu1 += t * (c3 * (c2 - c1) * c.il2 + c2 * (c3 - c1) * c.il3);
            mu2 += t * (c3 * (c1 - c2) * c.il1 + c1 * (c3 - c2) * c.il3);
            mu3 += t * (c2 * (c1 - c3) * c.il1 + c1 * (c2 - c3) * c.il2);
        }
    }
    b.muf[i] = mu1;
    b.muf[g.npad + i] = mu2;
    b.muf[2 * g.npad + i] = mu3;
}

// -------------------------------------------------- macroscopic state of a node
template <typename R>
struct Macro3 {
    R c1, c2, rho, itg, mu1, mu2, mu3, u[3], p, gr[3], F[3], am;
    unsigned walls;   // bit k: neighbour along e_k is a wall
};

// Gradients with the symmetric ghost of Eq. 43 (Eq. 20a), Laplacians of mu
// (Eq. 20b), F_s (potential form), G = rho g, u (Eq. 13b), the interfacial
// coefficient of Eq. 12 and p (Eq. 13c; c_s^2 / (1 - w_0) = 1/2 and
// s_0(u) = -u.u/2 on D3Q19).
template <typename R>
__device__ __forceinline__ Macro3<R> macro3(const Grid3& g, const Consts3<R>& c, const Bufs3<R>& b,
                                            const Nb3& nb, long long i, const R* gg) {
    Macro3<R> o;
    o.c1 = b.cf[i];
    o.c2 = b.cf[g.npad + i];
    o.mu1 = b.muf[i];
    o.mu2 = b.muf[g.npad + i];
    o.mu3 = b.muf[2 * g.npad + i];
    R g1[3] = {R(0), R(0), R(0)}, g2[3] = {R(0), R(0), R(0)};
    R lm1 = R(0), lm2 = R(0);
    o.walls = 0u;
#pragma unroll
    for (int k = 1; k < kQ; ++k) {
        const long long j = nb.at(EX[k], EY[k], EZ[k]);
        const bool wall = b.mat[j] != 0;
        o.walls |= wall ? 1u << k : 0u;
        const R v1 = wall ? o.c1 : b.cf[j];
        const R v2 = wall ? o.c2 : b.cf[g.npad + j];
        const R w1 = wall ? o.mu1 : b.muf[j];
        const R w2 = wall ? o.mu2 : b.muf[g.npad + j];
        const R w = wq<R>(k);
        if (EX[k]) { g1[0] += w * R(EX[k]) * v1; g2[0] += w * R(EX[k]) * v2; }
        if (EY[k]) { g1[1] += w * R(EY[k]) * v1; g2[1] += w * R(EY[k]) * v2; }
        if (EZ[k]) { g1[2] += w * R(EZ[k]) * v1; g2[2] += w * R(EZ[k]) * v2; }
        lm1 += w * (w1 - o.mu1);
        lm2 += w * (w2 - o.mu2);
    }
    lm1 *= R(6);
    lm2 *= R(6);
    const R grav[3] = {c.gx, c.gy, c.gz};
    o.rho = c.rho3 + c.drho1 * o.c1 + c.drho2 * o.c2;
    const R nu = c.nu3 + c.dnu1 * o.c1 + c.dnu2 * o.c2;
    o.itg = R(1) / (R(3) * nu + R(0.5));
    R m[3] = {R(0), R(0), R(0)}, sum = R(0);
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        if (EX[k]) m[0] += R(EX[k]) * gg[k];
        if (EY[k]) m[1] += R(EY[k]) * gg[k];
        if (EZ[k]) m[2] += R(EZ[k]) * gg[k];
        if (k) sum += gg[k];
    }
    const R irho = R(1) / o.rho;
    R udr = R(0), uu = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g1[a] *= R(3);
        g2[a] *= R(3);
        const R g3 = -(g1[a] + g2[a]);
        o.gr[a] = c.drho1 * g1[a] + c.drho2 * g2[a];
        o.F[a] = o.mu1 * g1[a] + o.mu2 * g2[a] + o.mu3 * g3 + o.rho * grav[a];
        o.u[a] = (m[a] + R(0.5) * o.F[a]) * irho;
        udr += o.u[a] * o.gr[a];
        uu += o.u[a] * o.u[a];
    }
    o.am = c.am1 * lm1 + c.am2 * lm2;
    o.p = R(0.5) * (sum + R(0.5) * udr - R(0.5) * o.rho * uu);
    return o;
}

// ------------------------------------------------------------------ collision
template <typename R>
__global__ __launch_bounds__(256) void col3_kernel(Grid3 g, Consts3<R> c, Bufs3<R> b, int cur) {
    const Node nd = node_of(g);
    if (!nd.in) return;
    const Nb3 nb = make_nb3(g, nd.x, nd.y, nd.z);
    const long long i = nb.at(0, 0, 0);
    if (b.mat[i]) return;
    const R* __restrict__ P = b.pop[cur];
    R* __restrict__ Q = b.pop[cur ^ 1];
    R f1[kQ], f2[kQ], gg[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        const long long j = nb.at(-EX[k], -EY[k], -EZ[k]);
        f1[k] = P[k * g.npad + j];
        f2[k] = P[(kQ + k) * g.npad + j];
        gg[k] = P[(2 * kQ + k) * g.npad + j];
    }
    const Macro3<R> o = macro3<R>(g, c, b, nb, i, gg);
    R ho[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) ho[q] = b.hist[q * g.npad + i];
    b.hist[i] = o.c1;
    b.hist[g.npad + i] = o.c2;
#pragma unroll
    for (int a = 0; a < 3; ++a) b.hist[(2 + a) * g.npad + i] = o.u[a];
    // Euler time derivative of c_i u (Eq. 19 inside Eq. 11a)
    R D1[3], D2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        D1[a] = o.c1 * o.u[a] - ho[0] * ho[2 + a];
        D2[a] = o.c2 * o.u[a] - ho[1] * ho[2 + a];
    }
    // BGK collision (Eq. 45) with the equilibria of Eqs. 2, 4 and the sources
    // of Eq. 11 (F_a outside the 1 - 1/(2 tau_g) factor), regrouped:
    //   f'^i_k = (1 - 1/tau_i) f^i_k + w_k (P_i + e_k.V_i),  k != 0
    //   g'_k = (1 - 1/tau_g) g_k + w_k (3 p / tau_g + e_k.G1 - G0)
    //          + s_k (rho / tau_g + fsg (e_k.A - u.A))
    const R em1 = c.eta1 * o.mu1, em2 = c.eta2 * o.mu2;
    const R fsg = R(1) - R(0.5) * o.itg;
    const R om1 = R(1) - c.itau1, om2 = R(1) - c.itau2, omg = R(1) - o.itg;
    const R P1 = c.itau1 * em1, P2 = c.itau2 * em2;
    R V1[3], V2[3], A[3], G1[3];
    R uA = R(0), uF = R(0), uu = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        V1[a] = R(3) * (c.itau1 * o.c1 * o.u[a] + c.fs1 * D1[a]);
        V2[a] = R(3) * (c.itau2 * o.c2 * o.u[a] + c.fs2 * D2[a]);
        A[a] = o.gr[a] + R(3) * o.F[a];
        G1[a] = R(3) * (fsg * o.F[a] + o.u[a] * o.am);
        uA += o.u[a] * A[a];
        uF += o.u[a] * o.F[a];
        uu += o.u[a] * o.u[a];
    }
    const R G0 = R(3) * fsg * uF;
    const R Pg = R(3) * o.itg * o.p;
    const R Rg = o.itg * o.rho;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        const R w = wq<R>(k);
        const R eu = R(EX[k]) * o.u[0] + R(EY[k]) * o.u[1] + R(EZ[k]) * o.u[2];
        const R sk = w * (eu * (R(3) + R(4.5) * eu) - R(1.5) * uu);     // Eq. 4
        if (k == 0) {
            f1[0] = om1 * f1[0] + c.itau1 * (o.c1 + (w - R(1)) * em1);
            f2[0] = om2 * f2[0] + c.itau2 * (o.c2 + (w - R(1)) * em2);
            gg[0] = omg * gg[0] + (w - R(1)) * Pg + sk * (Rg - fsg * uA) - w * G0;
        } else {
            const R eV1 = R(EX[k]) * V1[0] + R(EY[k]) * V1[1] + R(EZ[k]) * V1[2];
            const R eV2 = R(EX[k]) * V2[0] + R(EY[k]) * V2[1] + R(EZ[k]) * V2[2];
            const R eA = R(EX[k]) * A[0] + R(EY[k]) * A[1] + R(EZ[k]) * A[2];
            const R eG = R(EX[k]) * G1[0] + R(EY[k]) * G1[1] + R(EZ[k]) * G1[2];
            f1[k] = om1 * f1[k] + w * (P1 + eV1);
            f2[k] = om2 * f2[k] + w * (P2 + eV2);
            gg[k] = omg * gg[k] + w * (Pg + eG - G0) + sk * (Rg + fsg * (eA - uA));
        }
        Q[k * g.npad + i] = f1[k];
        Q[(kQ + k) * g.npad + i] = f2[k];
        Q[(2 * kQ + k) * g.npad + i] = gg[k];
    }
    if (o.walls) {
#pragma unroll
        for (int k = 1; k < kQ; ++k) {
            if (!((o.walls >> k) & 1u)) continue;
            const long long j = nb.at(EX[k], EY[k], EZ[k]);
            const double* t = &b.mtab[kMatStride * b.mat[j]];
            // moving-wall term -2 w_k a e_k.u_w / c_s^2 (wall velocity in x-y)
            const R corr = -R(6) * wq<R>(k) * (R(EX[k]) * R(t[3]) + R(EY[k]) * R(t[4]));
            const int ko = opp(k);
            Q[ko * g.npad + j] = f1[k] + corr * o.c1;
            Q[(kQ + ko) * g.npad + j] = f2[k] + corr * o.c2;
            Q[(2 * kQ + ko) * g.npad + j] = gg[k] + corr * o.rho;
        }
    }
}

// --------------------------------------------------------------------- init
template <typename R>
__global__ __launch_bounds__(256) void stage3_kernel(Grid3 g, Bufs3<R> b, const double* in5) {
    const Node p = node_of(g);
    if (!p.in) return;
    const long long i = ((long long)p.z * g.ny + p.y) * g.pitch + p.x;
    const long long hi = ((long long)p.z * g.ny + p.y) * g.nx + p.x;
    const long long n = (long long)g.nx * g.ny * g.nz;
    const bool fl = !b.mat[i];
    b.cf[i] = fl ? R(in5[hi]) : R(0);
    b.cf[g.npad + i] = fl ? R(in5[n + hi]) : R(0);
}

// Equilibrium populations (Eqs. 2, 4 with p = 0) written where each node
// pulls them in the first step (slot P_k[x - e_k]), history (c1, c2, u).
template <typename R>
__global__ __launch_bounds__(256) void init3_kernel(Grid3 g, Consts3<R> c, Bufs3<R> b,
                                                    const double* in5) {
    const Node p = node_of(g);
    if (!p.in) return;
    const Nb3 nb = make_nb3(g, p.x, p.y, p.z);
    const long long i = nb.at(0, 0, 0);
    const long long hi = ((long long)p.z * g.ny + p.y) * g.nx + p.x;
    const long long n = (long long)g.nx * g.ny * g.nz;
    if (b.mat[i]) {
#pragma unroll
        for (int q = 0; q < 5; ++q) b.hist[q * g.npad + i] = R(0);
        return;
    }
    const R c1 = b.cf[i], c2 = b.cf[g.npad + i];
    const R u[3] = {R(in5[2 * n + hi]), R(in5[3 * n + hi]), R(in5[4 * n + hi])};
    const R rho = c.rho3 + c.drho1 * c1 + c.drho2 * c2;
    const R em1 = c.eta1 * b.muf[i], em2 = c.eta2 * b.muf[g.npad + i];
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    R* Pd = b.pop[0];
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        const R w = wq<R>(k);
        const R eu = R(EX[k]) * u[0] + R(EY[k]) * u[1] + R(EZ[k]) * u[2];
        const R sk = w * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
        R fe1, fe2;
        if (k == 0) {
            fe1 = c1 + (w - R(1)) * em1;
            fe2 = c2 + (w - R(1)) * em2;
        } else {
            fe1 = w * (em1 + R(3) * c1 * eu);
            fe2 = w * (em2 + R(3) * c2 * eu);
        }
        const long long j = nb.at(-EX[k], -EY[k], -EZ[k]);
        Pd[k * g.npad + j] = fe1;
        Pd[(kQ + k) * g.npad + j] = fe2;
        Pd[(2 * kQ + k) * g.npad + j] = rho * sk;
    }
    b.hist[i] = c1;
    b.hist[g.npad + i] = c2;
#pragma unroll
    for (int a = 0; a < 3; ++a) b.hist[(2 + a) * g.npad + i] = u[a];
}

// ------------------------------------------------------------------ readout
template <typename R>
__global__ __launch_bounds__(256) void read3_kernel(Grid3 g, Consts3<R> c, Bufs3<R> b, int cur,
                                                    double* out) {
    const Node nd = node_of(g);
    if (!nd.in) return;
    const Nb3 nb = make_nb3(g, nd.x, nd.y, nd.z);
    const long long i = nb.at(0, 0, 0);
    const long long hi = ((long long)nd.z * g.ny + nd.y) * g.nx + nd.x;
    const long long n = (long long)g.nx * g.ny * g.nz;
    if (b.mat[i]) {
        for (int f = 0; f < 11; ++f) out[f * n + hi] = 0.0;
        return;
    }
    const R* __restrict__ P = b.pop[cur];
    R gg[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) gg[k] = P[(2 * kQ + k) * g.npad + nb.at(-EX[k], -EY[k], -EZ[k])];
    const Macro3<R> o = macro3<R>(g, c, b, nb, i, gg);
    const double v[11] = {double(o.c1), double(o.c2), double(R(1) - o.c1 - o.c2), double(o.rho),
                          double(o.u[0]), double(o.u[1]), double(o.u[2]), double(o.p),
                          double(o.mu1), double(o.mu2), double(o.mu3)};
    for (int f = 0; f < 11; ++f) out[f * n + hi] = v[f];
}

// populations f(x) of family fam (19 planes), pulled; walls read 0
template <typename R>
__global__ __launch_bounds__(256) void pops3_kernel(Grid3 g, Bufs3<R> b, int cur, int fam,
                                                    double* out) {
    const Node nd = node_of(g);
    if (!nd.in) return;
    const Nb3 nb = make_nb3(g, nd.x, nd.y, nd.z);
    const long long i = nb.at(0, 0, 0);
    const long long hi = ((long long)nd.z * g.ny + nd.y) * g.nx + nd.x;
    const long long n = (long long)g.nx * g.ny * g.nz;
    const bool wall = b.mat[i] != 0;
    const R* __restrict__ P = b.pop[cur];
#pragma unroll
    for (int k = 0; k < kQ; ++k)
        out[k * n + hi] =
            wall ? 0.0 : double(P[(fam * kQ + k) * g.npad + nb.at(-EX[k], -EY[k], -EZ[k])]);
}

// -------------------------------------------------------------------- mass
// Deterministic two-pass sum of c1, c2, c3 over fluid nodes (pulled
// populations of buffer cur): block b sums a fixed range of nodes in a fixed
// order and tree; one block then adds the partials in order.
template <typename R>
__global__ __launch_bounds__(256) void mass3_partial_kernel(Grid3 g, Bufs3<R> b, int cur,
                                                            double* partials) {
    __shared__ double sm[3][256];
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long per = (n + kReduceBlocks - 1) / kReduceBlocks;
    const long long lo = per * blockIdx.x;
    const long long hi = lo + per < n ? lo + per : n;
    const R* __restrict__ P = b.pop[cur];
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (long long h = lo + threadIdx.x; h < hi; h += 256) {
        const int x = int(h % g.nx);
        const long long r = h / g.nx;
        const int y = int(r % g.ny), z = int(r / g.ny);
        const Nb3 nb = make_nb3(g, x, y, z);
        const long long i = nb.at(0, 0, 0);
        if (b.mat[i]) continue;
        double a = 0.0, c = 0.0;
#pragma unroll
        for (int k = 0; k < kQ; ++k) {
            const long long j = nb.at(-EX[k], -EY[k], -EZ[k]);
            a += double(P[k * g.npad + j]);
            c += double(P[(kQ + k) * g.npad + j]);
        }
        s1 += a;
        s2 += c;
        s3 += 1.0 - a - c;
    }
    sm[0][threadIdx.x] = s1;
    sm[1][threadIdx.x] = s2;
    sm[2][threadIdx.x] = s3;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (int(threadIdx.x) < st)
            for (int q = 0; q < 3; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 3) partials[blockIdx.x * 3 + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void mass3_final_kernel(const double* partials, double* out) {
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int b = 0; b < kReduceBlocks; ++b) s += partials[b * 3 + threadIdx.x];
        out[threadIdx.x] = s;
    }
    if (threadIdx.x == 3) {
        double s = 0.0;
        for (int b = 0; b < kReduceBlocks; ++b) s += partials[b * 3] + partials[b * 3 + 1];
        out[3] = (s == s && s - s == 0.0) ? 0.0 : 1.0;   // NaN/Inf flag
    }
}

dim3 grid_of(const Grid3& g) {
    return dim3((g.nx + kBlockX - 1) / kBlockX, (g.ny + kBlockY - 1) / kBlockY, g.nz);
}

template <typename R>
hipError_t step_r(const Grid3& g, const void* consts, const void* bufs, int cur, hipStream_t s) {
    const Consts3<R>& c = *static_cast<const Consts3<R>*>(consts);
    const Bufs3<R>& b = *static_cast<const Bufs3<R>*>(bufs);
    const dim3 gr = grid_of(g);
    hipLaunchKernelGGL((c3_kernel<R>), gr, dim3(256), 0, s, g, b, cur);
    hipLaunchKernelGGL((mu3_kernel<R>), gr, dim3(256), 0, s, g, c, b);
    hipLaunchKernelGGL((col3_kernel<R>), gr, dim3(256), 0, s, g, c, b, cur);
    return hipGetLastError();
}

template <typename R>
hipError_t c_mu_r(const Grid3& g, const void* consts, const void* bufs, int cur, hipStream_t s) {
    const Consts3<R>& c = *static_cast<const Consts3<R>*>(consts);
    const Bufs3<R>& b = *static_cast<const Bufs3<R>*>(bufs);
    const dim3 gr = grid_of(g);
    hipLaunchKernelGGL((c3_kernel<R>), gr, dim3(256), 0, s, g, b, cur);
    hipLaunchKernelGGL((mu3_kernel<R>), gr, dim3(256), 0, s, g, c, b);
    return hipGetLastError();
}

template <typename R>
hipError_t init_r(const Grid3& g, const void* consts, const void* bufs, const double* in5,
                  hipStream_t s) {
    const Consts3<R>& c = *static_cast<const Consts3<R>*>(consts);
    const Bufs3<R>& b = *static_cast<const Bufs3<R>*>(bufs);
    const dim3 gr = grid_of(g);
    hipLaunchKernelGGL((stage3_kernel<R>), gr, dim3(256), 0, s, g, b, in5);
    hipLaunchKernelGGL((mu3_kernel<R>), gr, dim3(256), 0, s, g, c, b);
    hipLaunchKernelGGL((init3_kernel<R>), gr, dim3(256), 0, s, g, c, b, in5);
    return hipGetLastError();
}

template <typename R>
hipError_t read_r(const Grid3& g, const void* consts, const void* bufs, int cur, double* out,
                  hipStream_t s) {
    hipError_t e = c_mu_r<R>(g, consts, bufs, cur, s);
    if (e != hipSuccess) return e;
    const Consts3<R>& c = *static_cast<const Consts3<R>*>(consts);
    const Bufs3<R>& b = *static_cast<const Bufs3<R>*>(bufs);
    hipLaunchKernelGGL((read3_kernel<R>), grid_of(g), dim3(256), 0, s, g, c, b, cur, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch3_step(int prec, const Grid3& g, const void* consts, const void* bufs, int cur,
                        hipStream_t s) {
    return prec == 0 ? step_r<double>(g, consts, bufs, cur, s)
                     : step_r<float>(g, consts, bufs, cur, s);
}

hipError_t launch3_c_mu(int prec, const Grid3& g, const void* consts, const void* bufs, int cur,
                        hipStream_t s) {
    return prec == 0 ? c_mu_r<double>(g, consts, bufs, cur, s)
                     : c_mu_r<float>(g, consts, bufs, cur, s);
}

hipError_t launch3_init(int prec, const Grid3& g, const void* consts, const void* bufs,
                        const double* in5, hipStream_t s) {
    return prec == 0 ? init_r<double>(g, consts, bufs, in5, s)
                     : init_r<float>(g, consts, bufs, in5, s);
}

hipError_t launch3_readout(int prec, const Grid3& g, const void* consts, const void* bufs,
                           int cur, double* out11, hipStream_t s) {
    return prec == 0 ? read_r<double>(g, consts, bufs, cur, out11, s)
                     : read_r<float>(g, consts, bufs, cur, out11, s);
}

hipError_t launch3_populations(int prec, const Grid3& g, const void* bufs, int cur, int fam,
                               double* out19, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL((pops3_kernel<double>), grid_of(g), dim3(256), 0, s, g,
                           *static_cast<const Bufs3<double>*>(bufs), cur, fam, out19);
    else
        hipLaunchKernelGGL((pops3_kernel<float>), grid_of(g), dim3(256), 0, s, g,
                           *static_cast<const Bufs3<float>*>(bufs), cur, fam, out19);
    return hipGetLastError();
}

hipError_t launch3_mass(int prec, const Grid3& g, const void* bufs, int cur, double* partials,
                        double* result, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL((mass3_partial_kernel<double>), dim3(kReduceBlocks), dim3(256), 0, s,
                           g, *static_cast<const Bufs3<double>*>(bufs), cur, partials);
    else
        hipLaunchKernelGGL((mass3_partial_kernel<float>), dim3(kReduceBlocks), dim3(256), 0, s,
                           g, *static_cast<const Bufs3<float>*>(bufs), cur, partials);
    hipLaunchKernelGGL(mass3_final_kernel, dim3(1), dim3(64), 0, s, partials, result);
    return hipGetLastError();
}

}  // namespace tlb3
