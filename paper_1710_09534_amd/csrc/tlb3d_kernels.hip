// tlb3d_kernels.hip -- gfx950 kernels of the three-dimensional (D3Q19)
// version of the ternary wetting lattice Boltzmann step (Liang et al.,
// arXiv:1710.09534; the model is stated on D2Q9 "without loss of
// generality", Sec. II.A, and carried to D3Q19 link by link).
//
// One step is two launches:
//   c3_kernel     pulls f^1, f^2 (38 planes) and stores c1, c2 (Eqs. 3, 13a);
//   fused3_kernel marches 64 x 4 tiles along z: forms the chemical
//                 potentials in LDS from c with the wetting ghosts of Eq. 42
//                 across wall links (Eqs. 8, 20b; Eq. 6 for lambda > 0), then
//                 pulls all 57 populations, forms gradients with the symmetric
//                 ghosts of Eq. 43, forces, velocity, interfacial force,
//                 pressure and the Euler time derivative (Eqs. 12-15, 18b, 19),
//                 collides (Eqs. 2, 4, 11, 45) and stores the 57 post-collision
//                 populations, with half-way bounce-back (Eq. 44) folded into
//                 the stores: a fluid node whose neighbour x + e_k is a wall
//                 writes f'_k(x) (plus the moving-wall term) into slot
//                 P_opp(k) of that wall node, the slot only x pulls from.
// c needs a radius-2 halo in every direction; splitting at c (2 values per
// node through HBM) costs far less than recomputing that halo from the
// populations of a 3-D tile.  mu3_kernel (global mu) serves init and readout.
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
// s_0(u) = -u.u/2 on D3Q19).  N supplies, for link k, whether the neighbour
// is a wall and its c1, c2, mu1, mu2.
// 1/x: FP32 arithmetic uses the hardware reciprocal (1 ulp), FP64 divides
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename R, class N>
__device__ __forceinline__ Macro3<R> macro_core(const Consts3<R>& c, R c1, R c2, R mu1, R mu2,
                                                R mu3, const N& nbv, const R* gg) {
    Macro3<R> o;
    o.c1 = c1;
    o.c2 = c2;
    o.mu1 = mu1;
    o.mu2 = mu2;
    o.mu3 = mu3;
    R g1[3] = {R(0), R(0), R(0)}, g2[3] = {R(0), R(0), R(0)};
    R lm1 = R(0), lm2 = R(0);
    o.walls = 0u;
#pragma unroll
    for (int k = 1; k < kQ; ++k) {
        const bool wall = nbv.wall(k);
        o.walls |= wall ? 1u << k : 0u;
        const R v1 = wall ? c1 : nbv.c1(k);
        const R v2 = wall ? c2 : nbv.c2(k);
        const R w1 = wall ? mu1 : nbv.mu1(k);
        const R w2 = wall ? mu2 : nbv.mu2(k);
        const R w = wq<R>(k);
        if (EX[k]) { g1[0] += w * R(EX[k]) * v1; g2[0] += w * R(EX[k]) * v2; }
        if (EY[k]) { g1[1] += w * R(EY[k]) * v1; g2[1] += w * R(EY[k]) * v2; }
        if (EZ[k]) { g1[2] += w * R(EZ[k]) * v1; g2[2] += w * R(EZ[k]) * v2; }
        lm1 += w * (w1 - mu1);
        lm2 += w * (w2 - mu2);
    }
    lm1 *= R(6);
    lm2 *= R(6);
    const R grav[3] = {c.gx, c.gy, c.gz};
    o.rho = c.rho3 + c.drho1 * c1 + c.drho2 * c2;
    const R nu = c.nu3 + c.dnu1 * c1 + c.dnu2 * c2;
    o.itg = recip(R(3) * nu + R(0.5));
    R m[3] = {R(0), R(0), R(0)}, sum = R(0);
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        if (EX[k]) m[0] += R(EX[k]) * gg[k];
        if (EY[k]) m[1] += R(EY[k]) * gg[k];
        if (EZ[k]) m[2] += R(EZ[k]) * gg[k];
        if (k) sum += gg[k];
    }
    const R irho = recip(o.rho);
    R udr = R(0), uu = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g1[a] *= R(3);
        g2[a] *= R(3);
        const R g3 = -(g1[a] + g2[a]);
        o.gr[a] = c.drho1 * g1[a] + c.drho2 * g2[a];
        o.F[a] = mu1 * g1[a] + mu2 * g2[a] + mu3 * g3 + o.rho * grav[a];
        o.u[a] = (m[a] + R(0.5) * o.F[a]) * irho;
        udr += o.u[a] * o.gr[a];
        uu += o.u[a] * o.u[a];
    }
    o.am = c.am1 * lm1 + c.am2 * lm2;
    o.p = R(0.5) * (sum + R(0.5) * udr - R(0.5) * o.rho * uu);
    return o;
}

// neighbour values from the global c and mu fields (readout)
template <typename R>
struct GlobalNbr {
    const Grid3& g;
    const Bufs3<R>& b;
    const Nb3& nb;
    __device__ __forceinline__ long long j(int k) const { return nb.at(EX[k], EY[k], EZ[k]); }
    __device__ __forceinline__ bool wall(int k) const { return b.mat[j(k)] != 0; }
    __device__ __forceinline__ R c1(int k) const { return b.cf[j(k)]; }
    __device__ __forceinline__ R c2(int k) const { return b.cf[g.npad + j(k)]; }
    __device__ __forceinline__ R mu1(int k) const { return b.muf[j(k)]; }
    __device__ __forceinline__ R mu2(int k) const { return b.muf[g.npad + j(k)]; }
};

// ------------------------------------------------------- fused mu + collision
// The step kernel proper.  A block owns a 64 x 4 tile of (x, y) and marches
// along z over a chunk of planes.  LDS holds a ring of five c planes (tile +
// radius-2 halo, with the material bytes) and a ring of three mu planes
// (tile + radius-1 halo).  Per plane z: the block loads c of plane z+2 from
// the c field, forms mu of plane z+1 (Eqs. 8, 20b with the wetting ghosts of
// Eq. 42; Eq. 6 for lambda > 0), then each thread collides its node of plane
// z with gradients and Laplacians read from the rings.  The 57 pulls of a
// node are issued before the plane's LDS work so that they are in flight
// while it runs.  Populations are addressed through one buffer resource per
// family (plane offset in the scalar offset, node offset in a 32-bit lane
// offset).
constexpr int kRW = kBlockX + 4;   // c ring columns x0-2 .. x0+65
constexpr int kRH = kBlockY + 4;   // c ring rows    y0-2 .. y0+5
constexpr int kMW = kBlockX + 2;   // mu ring columns x0-1 .. x0+64
constexpr int kMH = kBlockY + 2;   // mu ring rows    y0-1 .. y0+4
constexpr int kZChunk = 32;        // z planes per block
constexpr int kCPer = (kRH * kRW + 255) / 256;   // c ring positions per thread

// Order of the c fetch of plane z+2 and the 57 pulls of plane z.  Vector
// loads retire in order, so waiting for c fetched after the pulls waits for
// every pull too, and the pulls' latency is not hidden behind the LDS work
// of the plane.  FP64 (one workgroup per CU) fetches c first and gains
// 7 % per step; FP32 keeps the fetch after the pulls: staging c in
// registers across the pulls costs it spills at 3 waves per SIMD or a
// fourth of its occupancy at 2, and its three workgroups per CU already
// overlap each other's loads (measured: 1.45 ms per step at 192 x 192 x 256
// against 1.49-1.52 ms with the early fetch).
template <typename R>
constexpr bool kEarlyC = sizeof(R) == 8;

// The Laplacians of mu_plane: FP64 sums over the ring values without a
// branch per link and repeats the sum with the wetting ghosts only at nodes
// with a wall link (fused3<double> -8 % per step; the compiler may contract
// the two forms differently, so results agree to rounding).  In FP32 the
// branch-free form spills 4 VGPRs at 3 waves per SIMD and is 2 % slower.
template <typename R>
constexpr bool kFlatMu = sizeof(R) == 8;

// c1, c2 and material of up to kCPer ring positions of one thread
template <typename R>
struct CStage {
    uint8_t m[kCPer];
    R c1[kCPer], c2[kCPer];
};

template <typename R>
struct Ring3 {
    R c[5][2][kRH * kRW];
    R mu[3][3][kMH * kMW];
    R mt[kMatStride * (kMaxMaterials + 1)];
    uint8_t m[5][kRH * kRW];
};

using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, gfx9 family
// a lane offset past every resource (a family of 19 planes stays below
// 2^31 bytes): loads from it return 0, stores to it are dropped
constexpr unsigned kDiscard3 = 0x80000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), kRsrcWord3);
}

template <typename R>
__device__ __forceinline__ R bload(rsrc_t r, unsigned vo, unsigned so) {
    if constexpr (sizeof(R) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(vo), int(so), 0));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(vo), int(so), 0));
}

// FP32 population stores are non-temporal (cache-policy operand bit 1):
// written once per step and read once in the next, they then no longer evict
// the halo lines that neighbouring tiles re-read from L2 (measured: 7 % less
// step time in FP32; FP64 is 4 % slower with it and keeps the default).
template <typename R>
__device__ __forceinline__ void bstore(rsrc_t r, unsigned vo, unsigned so, R v) {
    if constexpr (sizeof(R) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r,
            int(vo), int(so), 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, int(vo), int(so), 2);
}

// neighbour values from the LDS rings: pointers of the node's position in
// the c / mu planes z-1, z, z+1
template <typename R>
struct RingNbr {
    const R* c1p[3];
    const R* c2p[3];
    const uint8_t* mp[3];
    const R* m1p[3];
    const R* m2p[3];
    __device__ __forceinline__ bool wall(int k) const { return mp[EZ[k] + 1][EY[k] * kRW + EX[k]] != 0; }
    __device__ __forceinline__ R c1(int k) const { return c1p[EZ[k] + 1][EY[k] * kRW + EX[k]]; }
    __device__ __forceinline__ R c2(int k) const { return c2p[EZ[k] + 1][EY[k] * kRW + EX[k]]; }
    __device__ __forceinline__ R mu1(int k) const { return m1p[EZ[k] + 1][EY[k] * kMW + EX[k]]; }
    __device__ __forceinline__ R mu2(int k) const { return m2p[EZ[k] + 1][EY[k] * kMW + EX[k]]; }
};

__device__ __forceinline__ int cslot(int zz, int z0) { return (zz - z0 + 10) % 5; }
__device__ __forceinline__ int mslot(int zz, int z0) { return (zz - z0 + 9) % 3; }

// FP32: at most 168 VGPRs (3 waves per SIMD) fits without spills and runs
// faster than the 2 waves the compiler picks by itself; FP64 needs its 256.
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 1 : 3)))
void fused3_kernel(Grid3 g, Consts3<R> c, Bufs3<R> b, int cur) {
    __shared__ Ring3<R> sm;
    const int tx = int(threadIdx.x % kBlockX), ty = int(threadIdx.x / kBlockX);
    const int x0 = blockIdx.x * kBlockX, y0 = blockIdx.y * kBlockY;
    const int z0 = blockIdx.z * kZChunk;
    const int z1 = z0 + kZChunk < g.nz ? z0 + kZChunk : g.nz;
    const int x = x0 + tx, y = y0 + ty;
    const bool own = x < g.nx && y < g.ny;
    for (int q = threadIdx.x; q < kMatStride * (kMaxMaterials + 1); q += 256) sm.mt[q] = R(b.mtab[q]);

    const unsigned ps = unsigned(g.npad * (long long)sizeof(R));   // plane bytes
    rsrc_t src[3], dst[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        src[f] = make_rsrc(b.pop[cur] + f * kQ * g.npad, unsigned(kQ) * ps);
        dst[f] = make_rsrc(b.pop[cur ^ 1] + f * kQ * g.npad, unsigned(kQ) * ps);
    }

    // c and material of plane zz (tile + radius-2 halo) into its ring slot:
    // load_c in one pass, or fetch_c into registers (at most kCPer positions
    // per thread) and put_c later.  fetch_c issues every load on every lane
    // (a lane past the ring re-reads a valid position and does not store
    // it), so that the wait counts do not depend on control flow.  (Lambdas
    // capture by value: taking the address of the by-value kernel arguments
    // would move them to private memory.)
    auto fetch_c = [=](int zz, CStage<R>& st) {
        const long long zb = (long long)wrap(zz, g.nz) * g.ny;
#pragma unroll
        for (int it = 0; it < kCPer; ++it) {
            int q = int(threadIdx.x) + 256 * it;
            if (q >= kRH * kRW) q -= 256;
            const int r = q / kRW, col = q - r * kRW;
            const long long i = (zb + wrap(y0 - 2 + r, g.ny)) * g.pitch + wrap(x0 - 2 + col, g.nx);
            st.m[it] = b.mat[i];
            st.c1[it] = b.cf[i];
            st.c2[it] = b.cf[g.npad + i];
        }
    };
    auto load_c = [=](int zz) {
        const int sl = cslot(zz, z0);
        const long long zb = (long long)wrap(zz, g.nz) * g.ny;
        for (int q = threadIdx.x; q < kRH * kRW; q += 256) {
            const int r = q / kRW, col = q - r * kRW;
            const long long i = (zb + wrap(y0 - 2 + r, g.ny)) * g.pitch + wrap(x0 - 2 + col, g.nx);
            sm.m[sl][q] = b.mat[i];
            sm.c[sl][0][q] = b.cf[i];
            sm.c[sl][1][q] = b.cf[g.npad + i];
        }
    };
    auto put_c = [=](int zz, const CStage<R>& st) {
        const int sl = cslot(zz, z0);
#pragma unroll
        for (int it = 0; it < kCPer; ++it) {
            const int q = int(threadIdx.x) + 256 * it;
            if (q < kRH * kRW) {
                sm.m[sl][q] = st.m[it];
                sm.c[sl][0][q] = st.c1[it];
                sm.c[sl][1][q] = st.c2[it];
            }
        }
    };
    // mu of plane zz on the tile + radius-1 halo into its ring slot
    auto mu_plane = [=](int zz) {
        const int ms = mslot(zz, z0);
        const int s3[3] = {cslot(zz - 1, z0), cslot(zz, z0), cslot(zz + 1, z0)};
        for (int q = threadIdx.x; q < kMH * kMW; q += 256) {
            const int r = q / kMW, col = q - r * kMW;
            const int cq = (r + 1) * kRW + col + 1;
            R mu1 = R(0), mu2 = R(0), mu3 = R(0);
            if (!sm.m[s3[1]][cq]) {
                const R c1 = sm.c[s3[1]][0][cq], c2 = sm.c[s3[1]][1][cq], c3 = R(1) - c1 - c2;
                // Laplacians (Eq. 20b), with the ghost of Eq. 42 across a wall
                // link (wall value c(x))
                R l1 = R(0), l2 = R(0), l3 = R(0);
                auto lap_wet = [&]() {
                    l1 = l2 = l3 = R(0);
#pragma unroll
                    for (int k = 1; k < kQ; ++k) {
                        const int sl = s3[EZ[k] + 1];
                        const int nq = cq + EY[k] * kRW + EX[k];
                        const int m = sm.m[sl][nq];
                        R n1, n2, n3;
                        if (m) {
                            const R* t = &sm.mt[kMatStride * m];
                            n1 = c1 + c.k4D * (t[1] * c1 * c3 + t[0] * c1 * c2);
                            n2 = c2 + c.k4D * (-t[0] * c1 * c2 + t[2] * c2 * c3);
                            n3 = c3 + c.k4D * (-t[2] * c2 * c3 - t[1] * c1 * c3);
                        } else {
                            n1 = sm.c[sl][0][nq];
                            n2 = sm.c[sl][1][nq];
                            n3 = R(1) - n1 - n2;
                        }
                        l1 += wq<R>(k) * (n1 - c1);
                        l2 += wq<R>(k) * (n2 - c2);
                        l3 += wq<R>(k) * (n3 - c3);
                    }
                };
                if constexpr (kFlatMu<R>) {
                    // over the ring values without a branch per link; a node
                    // with a wall link takes them again with the ghosts
                    unsigned walls = 0u;
#pragma unroll
                    for (int k = 1; k < kQ; ++k) {
                        const int sl = s3[EZ[k] + 1];
                        const int nq = cq + EY[k] * kRW + EX[k];
                        walls |= sm.m[sl][nq];
                        const R n1 = sm.c[sl][0][nq], n2 = sm.c[sl][1][nq], n3 = R(1) - n1 - n2;
                        l1 += wq<R>(k) * (n1 - c1);
                        l2 += wq<R>(k) * (n2 - c2);
                        l3 += wq<R>(k) * (n3 - c3);
                    }
                    if (walls) lap_wet();
                } else {
                    lap_wet();
                }
                l1 *= R(6);
                l2 *= R(6);
                l3 *= R(6);
                const R tri = R(2) * c.lamT * c1 * c2 * c3;
                mu1 = c.k12D * (c.lam1 * c1 * (R(1) - c1) * (R(1) - R(2) * c1) - tri) - c.k34D * c.lam1 * l1;
                mu2 = c.k12D * (c.lam2 * c2 * (R(1) - c2) * (R(1) - R(2) * c2) - tri) - c.k34D * c.lam2 * l2;
                mu3 = c.k12D * (c.lam3 * c3 * (R(1) - c3) * (R(1) - R(2) * c3) - tri) - c.k34D * c.lam3 * l3;
                if (c.kB != R(0)) {   // lambda c1^2 c2^2 c3^2 term of Eq. 5 through Eq. 6
                    const R t = c.kB * c1 * c2 * c3;
                    mu1 += t * (c3 * (c2 - c1) * c.il2 + c2 * (c3 - c1) * c.il3);
                    mu2 += t * (c3 * (c1 - c2) * c.il1 + c1 * (c3 - c2) * c.il3);
                    mu3 += t * (c2 * (c1 - c3) * c.il1 + c1 * (c2 - c3) * c.il2);
                }
            }
            sm.mu[ms][0][q] = mu1;
            sm.mu[ms][1][q] = mu2;
            sm.mu[ms][2][q] = mu3;
        }
    };

    // prologue: c planes z0-2 .. z0+1, mu planes z0-1, z0
    for (int zz = z0 - 2; zz <= z0 + 1; ++zz) load_c(zz);
    __syncthreads();
    mu_plane(z0 - 1);
    mu_plane(z0);

    const int xs[3] = {wrap(x - 1, g.nx), x, wrap(x + 1, g.nx)};
    const int ys[3] = {wrap(y - 1, g.ny), y, wrap(y + 1, g.ny)};
    for (int z = z0; z < z1; ++z) {
        // pulls of this thread's node of plane z (issued before the LDS work)
        const int zs[3] = {wrap(z - 1, g.nz), z, wrap(z + 1, g.nz)};
        auto eidx = [=](int dx, int dy, int dz) -> unsigned {
            return unsigned(((long long)zs[dz + 1] * g.ny + ys[dy + 1]) * g.pitch + xs[dx + 1]);
        };
        const unsigned i = eidx(0, 0, 0);
        R f1[kQ], f2[kQ], gg[kQ];
        if constexpr (kEarlyC<R>) {
            CStage<R> next;
            fetch_c(z + 2, next);
            __builtin_amdgcn_sched_barrier(0);   // keep the c loads ahead of the pulls
            // Every lane issues every pull (a lane outside the lattice loads
            // from the discard offset, past the end of the resource, which
            // returns 0 without a memory access), so that the wait counts
            // before the ring stores do not depend on control flow.
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                const unsigned vo =
                    own ? eidx(-EX[k], -EY[k], -EZ[k]) * unsigned(sizeof(R)) : kDiscard3;
                f1[k] = bload<R>(src[0], vo, unsigned(k) * ps);
                f2[k] = bload<R>(src[1], vo, unsigned(k) * ps);
                gg[k] = bload<R>(src[2], vo, unsigned(k) * ps);
            }
            put_c(z + 2, next);
        } else {
#pragma unroll
            for (int k = 0; k < kQ; ++k) {
                const unsigned vo =
                    own ? eidx(-EX[k], -EY[k], -EZ[k]) * unsigned(sizeof(R)) : kDiscard3;
                f1[k] = bload<R>(src[0], vo, unsigned(k) * ps);
                f2[k] = bload<R>(src[1], vo, unsigned(k) * ps);
                gg[k] = bload<R>(src[2], vo, unsigned(k) * ps);
            }
            load_c(z + 2);
        }
        __syncthreads();
        mu_plane(z + 1);
        __syncthreads();
        if (!own) continue;
        const int cs = cslot(z, z0);
        const int cq = (ty + 2) * kRW + tx + 2;
        if (sm.m[cs][cq]) continue;
        const int mq = (ty + 1) * kMW + tx + 1;
        const int ms = mslot(z, z0);
        RingNbr<R> nbv;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int sl = cslot(z + d - 1, z0), ml = mslot(z + d - 1, z0);
            nbv.c1p[d] = &sm.c[sl][0][cq];
            nbv.c2p[d] = &sm.c[sl][1][cq];
            nbv.mp[d] = &sm.m[sl][cq];
            nbv.m1p[d] = &sm.mu[ml][0][mq];
            nbv.m2p[d] = &sm.mu[ml][1][mq];
        }
        const Macro3<R> o = macro_core<R>(c, sm.c[cs][0][cq], sm.c[cs][1][cq], sm.mu[ms][0][mq],
                                          sm.mu[ms][1][mq], sm.mu[ms][2][mq], nbv, gg);
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
        // BGK collision (Eq. 45) with the equilibria of Eqs. 2, 4 and the
        // sources of Eq. 11 (F_a outside the 1 - 1/(2 tau_g) factor), regrouped:
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
        const unsigned ob = i * unsigned(sizeof(R));
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
            bstore<R>(dst[0], ob, unsigned(k) * ps, f1[k]);
            bstore<R>(dst[1], ob, unsigned(k) * ps, f2[k]);
            bstore<R>(dst[2], ob, unsigned(k) * ps, gg[k]);
        }
        if (o.walls) {
#pragma unroll
            for (int k = 1; k < kQ; ++k) {
                if (!((o.walls >> k) & 1u)) continue;
                const int mn = nbv.mp[EZ[k] + 1][EY[k] * kRW + EX[k]];
                const R* t = &sm.mt[kMatStride * mn];
                // moving-wall term -2 w_k a e_k.u_w / c_s^2 (wall velocity in x-y)
                const R corr = -R(6) * wq<R>(k) * (R(EX[k]) * t[3] + R(EY[k]) * t[4]);
                const unsigned jb = eidx(EX[k], EY[k], EZ[k]) * unsigned(sizeof(R));
                const unsigned so = unsigned(opp(k)) * ps;
                bstore<R>(dst[0], jb, so, f1[k] + corr * o.c1);
                bstore<R>(dst[1], jb, so, f2[k] + corr * o.c2);
                bstore<R>(dst[2], jb, so, gg[k] + corr * o.rho);
            }
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
                                                    int za, int zb, double* out) {
    Node nd = node_of(g);                      // blockIdx.z counts planes from za
    nd.z += za;
    if (!nd.in || nd.z >= zb) return;
    const Nb3 nb = make_nb3(g, nd.x, nd.y, nd.z);
    const long long i = nb.at(0, 0, 0);
    const long long hi = ((long long)(nd.z - za) * g.ny + nd.y) * g.nx + nd.x;
    const long long n = (long long)g.nx * g.ny * (zb - za);
    if (b.mat[i]) {
        for (int f = 0; f < 11; ++f) out[f * n + hi] = 0.0;
        return;
    }
    const R* __restrict__ P = b.pop[cur];
    R gg[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) gg[k] = P[(2 * kQ + k) * g.npad + nb.at(-EX[k], -EY[k], -EZ[k])];
    const GlobalNbr<R> nbv{g, b, nb};
    const Macro3<R> o = macro_core<R>(c, b.cf[i], b.cf[g.npad + i], b.muf[i], b.muf[g.npad + i],
                                      b.muf[2 * g.npad + i], nbv, gg);
    const double v[11] = {double(o.c1), double(o.c2), double(R(1) - o.c1 - o.c2), double(o.rho),
                          double(o.u[0]), double(o.u[1]), double(o.u[2]), double(o.p),
                          double(o.mu1), double(o.mu2), double(o.mu3)};
    for (int f = 0; f < 11; ++f) out[f * n + hi] = v[f];
}

// populations f(x) of family fam (19 planes) on the planes [za, zb), pulled;
// walls read 0
template <typename R>
__global__ __launch_bounds__(256) void pops3_kernel(Grid3 g, Bufs3<R> b, int cur, int fam,
                                                    int za, int zb, double* out) {
    Node nd = node_of(g);
    nd.z += za;
    if (!nd.in || nd.z >= zb) return;
    const Nb3 nb = make_nb3(g, nd.x, nd.y, nd.z);
    const long long i = nb.at(0, 0, 0);
    const long long hi = ((long long)(nd.z - za) * g.ny + nd.y) * g.nx + nd.x;
    const long long n = (long long)g.nx * g.ny * (zb - za);
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
    hipLaunchKernelGGL((c3_kernel<R>), grid_of(g), dim3(256), 0, s, g, b, cur);
    const dim3 gf((g.nx + kBlockX - 1) / kBlockX, (g.ny + kBlockY - 1) / kBlockY,
                  (g.nz + kZChunk - 1) / kZChunk);
    hipLaunchKernelGGL((fused3_kernel<R>), gf, dim3(256), 0, s, g, c, b, cur);
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
hipError_t read_r(const Grid3& g, const void* consts, const void* bufs, int cur, int za, int zb,
                  double* out, hipStream_t s) {
    const Consts3<R>& c = *static_cast<const Consts3<R>*>(consts);
    const Bufs3<R>& b = *static_cast<const Bufs3<R>*>(bufs);
    dim3 gr = grid_of(g);
    gr.z = unsigned(zb - za);
    hipLaunchKernelGGL((read3_kernel<R>), gr, dim3(256), 0, s, g, c, b, cur, za, zb, out);
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
                           int cur, int za, int zb, double* out11, hipStream_t s) {
    if (za < 0 || zb > g.nz || za >= zb) return hipErrorInvalidValue;
    return prec == 0 ? read_r<double>(g, consts, bufs, cur, za, zb, out11, s)
                     : read_r<float>(g, consts, bufs, cur, za, zb, out11, s);
}

hipError_t launch3_populations(int prec, const Grid3& g, const void* bufs, int cur, int fam,
                               int za, int zb, double* out19, hipStream_t s) {
    if (za < 0 || zb > g.nz || za >= zb) return hipErrorInvalidValue;
    dim3 gr = grid_of(g);
    gr.z = unsigned(zb - za);
    if (prec == 0)
        hipLaunchKernelGGL((pops3_kernel<double>), gr, dim3(256), 0, s, g,
                           *static_cast<const Bufs3<double>*>(bufs), cur, fam, za, zb, out19);
    else
        hipLaunchKernelGGL((pops3_kernel<float>), gr, dim3(256), 0, s, g,
                           *static_cast<const Bufs3<float>*>(bufs), cur, fam, za, zb, out19);
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
