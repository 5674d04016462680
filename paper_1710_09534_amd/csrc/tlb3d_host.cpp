// tlb3d_host.cpp -- host runtime of the C ABI declared in include/tlb3d.h:
// parameter derivation and validation, workspace layout, launches and health
// checks of the three-dimensional (D3Q19) step.  All device work goes to the
// context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tlb3d.h"
#include "tlb3d_internal.h"

using namespace tlb3;

namespace {

thread_local std::string g_last_error3;

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout3 {
    int pitch;
    size_t npad, n;
    size_t stage_doubles;
    size_t off_pop[2], off_hist, off_cf, off_muf, off_mat, off_mtab, off_stage, off_part,
        off_result, total;
};

Layout3 make_layout3(int nx, int ny, int nz, int prec) {
    Layout3 L{};
    const size_t s = prec == 0 ? 8 : 4;
    L.pitch = int(align_up(size_t(nx), kBlockX));
    L.npad = size_t(L.pitch) * ny * nz;
    L.n = size_t(nx) * ny * nz;
    size_t o = 0;
    for (int b = 0; b < 2; ++b) {
        L.off_pop[b] = o;
        o += align_up(size_t(3 * kQ) * L.npad * s, kAlign);
    }
    L.off_hist = o; o += align_up(5 * L.npad * s, kAlign);
    L.off_cf = o; o += align_up(2 * L.npad * s, kAlign);
    L.off_muf = o; o += align_up(3 * L.npad * s, kAlign);
    L.off_mat = o; o += align_up(L.npad, kAlign);
    L.off_mtab = o; o += align_up(kMatStride * (kMaxMaterials + 1) * sizeof(double), kAlign);
    // staging: the 5 input fields of init; readout and population copies pass
    // through it in bands of z-planes (at least one plane of 19 populations)
    L.stage_doubles = std::max(5 * L.n, size_t(kQ) * nx * ny);
    L.off_stage = o; o += align_up(L.stage_doubles * sizeof(double), kAlign);
    L.off_part = o; o += align_up(kReduceBlocks * 3 * sizeof(double), kAlign);
    L.off_result = o; o += kAlign;
    L.total = o;
    return L;
}

}  // namespace

struct tlb3_ctx {
    int nx, ny, nz, prec;
    tlb_fluid fl;
    double gz;
    Layout3 L;
    Grid3 grid;
    char* ws;
    hipStream_t stream;
    Consts3<double> c64;
    Consts3<float> c32;
    Bufs3<double> b64;
    Bufs3<float> b32;
    double lambda[3], lambdaT, M[2], eta[2];
    double* health = nullptr;   // pinned: last health result (sum c1, c2, c3, NaN flag)
    bool health_pending = false;
    bool geometry = false, inited = false, diverged = false;
    int cur = 0;
    int64_t steps = 0, check_interval = 100, since_check = 0;
    std::string err;
};

namespace {

tlb_status fail(tlb3_ctx* c, tlb_status s, const std::string& m) {
    if (c) c->err = m;
    g_last_error3 = m;
    return s;
}

tlb_status dev_fail(tlb3_ctx* c, hipError_t e, const char* where) {
    return fail(c, TLB_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

const void* consts_ptr(const tlb3_ctx* c) {
    return c->prec == 0 ? static_cast<const void*>(&c->c64) : static_cast<const void*>(&c->c32);
}
const void* bufs_ptr(const tlb3_ctx* c) {
    return c->prec == 0 ? static_cast<const void*>(&c->b64) : static_cast<const void*>(&c->b32);
}

template <typename R>
void fill3(Consts3<R>& k, const tlb3_ctx* c) {
    const tlb_fluid& f = c->fl;
    k.drho1 = R(f.rho[0] - f.rho[2]);
    k.drho2 = R(f.rho[1] - f.rho[2]);
    k.rho3 = R(f.rho[2]);
    k.dnu1 = R(f.nu[0] - f.nu[2]);
    k.dnu2 = R(f.nu[1] - f.nu[2]);
    k.nu3 = R(f.nu[2]);
    k.itau1 = R(1.0 / f.tau1);
    k.itau2 = R(1.0 / f.tau2);
    k.fs1 = R(1.0 - 0.5 / f.tau1);
    k.fs2 = R(1.0 - 0.5 / f.tau2);
    k.eta1 = R(c->eta[0]);
    k.eta2 = R(c->eta[1]);
    k.am1 = R((f.rho[0] - f.rho[2]) * c->M[0]);
    k.am2 = R((f.rho[1] - f.rho[2]) * c->M[1]);
    k.lam1 = R(c->lambda[0]);
    k.lam2 = R(c->lambda[1]);
    k.lam3 = R(c->lambda[2]);
    k.lamT = R(c->lambdaT);
    k.k12D = R(12.0 / f.D);
    k.k34D = R(0.75 * f.D);
    k.k4D = R(4.0 / f.D);
    k.gx = R(f.gravity[0]);
    k.gy = R(f.gravity[1]);
    k.gz = R(c->gz);
    k.kB = R(8.0 * f.lambda * c->lambdaT / f.D);
    k.il1 = R(1.0 / c->lambda[0]);
    k.il2 = R(1.0 / c->lambda[1]);
    k.il3 = R(1.0 / c->lambda[2]);
}

template <typename R>
void fill_bufs(Bufs3<R>& b, tlb3_ctx* c) {
    b.pop[0] = reinterpret_cast<R*>(c->ws + c->L.off_pop[0]);
    b.pop[1] = reinterpret_cast<R*>(c->ws + c->L.off_pop[1]);
    b.hist = reinterpret_cast<R*>(c->ws + c->L.off_hist);
    b.cf = reinterpret_cast<R*>(c->ws + c->L.off_cf);
    b.muf = reinterpret_cast<R*>(c->ws + c->L.off_muf);
    b.mat = reinterpret_cast<const uint8_t*>(c->ws + c->L.off_mat);
    b.mtab = reinterpret_cast<const double*>(c->ws + c->L.off_mtab);
}

double* stage_ptr(tlb3_ctx* c) { return reinterpret_cast<double*>(c->ws + c->L.off_stage); }

tlb_status run_mass(tlb3_ctx* c) {
    hipError_t e = launch3_mass(c->prec, c->grid, bufs_ptr(c), c->cur,
                                reinterpret_cast<double*>(c->ws + c->L.off_part),
                                reinterpret_cast<double*>(c->ws + c->L.off_result), c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "mass reduction");
    return TLB_OK;
}

void poll_health(tlb3_ctx* c) {
    if (!c->health_pending) return;
    if (hipStreamQuery(c->stream) != hipSuccess) return;
    c->health_pending = false;
    if (c->health[3] != 0.0) c->diverged = true;
}

tlb_status step_impl(tlb3_ctx* c, int64_t nsteps, bool checks) {
    for (int64_t s = 0; s < nsteps; ++s) {
        hipError_t e = launch3_step(c->prec, c->grid, consts_ptr(c), bufs_ptr(c), c->cur, c->stream);
        if (e != hipSuccess) return dev_fail(c, e, "step kernels");
        c->cur ^= 1;
        ++c->steps;
        if (checks && c->check_interval > 0 && ++c->since_check >= c->check_interval) {
            c->since_check = 0;
            tlb_status st = run_mass(c);
            if (st != TLB_OK) return st;
            e = hipMemcpyAsync(c->health, c->ws + c->L.off_result, 4 * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream);
            if (e != hipSuccess) return dev_fail(c, e, "health copy");
            c->health_pending = true;
        }
    }
    return TLB_OK;
}

}  // namespace

extern "C" {

// the fused step kernel addresses each family of 19 planes as one buffer
// resource with 32-bit sizes and offsets
static bool fits_offsets3(const Layout3& L, int p) {
    return size_t(kQ) * L.npad * (p == 0 ? 8 : 4) < (size_t(1) << 31);
}

size_t tlb3_workspace_bytes(int nx, int ny, int nz, tlb_precision p) {
    if (nx < 3 || ny < 3 || nz < 3 || nz > 65535 || (p != TLB_FP64 && p != TLB_FP32)) return 0;
    const Layout3 L = make_layout3(nx, ny, nz, int(p));
    return fits_offsets3(L, int(p)) ? L.total : 0;
}

tlb_status tlb3_create(int nx, int ny, int nz, tlb_precision p, const tlb_fluid* fl,
                       double gravity_z, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                       tlb3_ctx** out) {
    if (!out) return fail(nullptr, TLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!fl || !dev_workspace) return fail(nullptr, TLB_EINVAL, "null fluid or workspace");
    if (nx < 3 || ny < 3 || nz < 3) return fail(nullptr, TLB_EINVAL, "nx, ny and nz must be >= 3");
    if (nz > 65535) return fail(nullptr, TLB_EINVAL, "nz must be <= 65535");
    if (p != TLB_FP64 && p != TLB_FP32)
        return fail(nullptr, TLB_EINVAL, "the 3-D step stores FP64 or FP32 populations");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign)
        return fail(nullptr, TLB_EINVAL, "workspace must be 256-byte aligned");
    const Layout3 L = make_layout3(nx, ny, nz, int(p));
    if (!fits_offsets3(L, int(p)))
        return fail(nullptr, TLB_EINVAL, "lattice too large: a family of 19 planes must stay below 2 GiB");
    if (ws_bytes < L.total) return fail(nullptr, TLB_ENOMEM, "workspace too small");
    double lam[3] = {fl->sigma12 + fl->sigma13 - fl->sigma23, fl->sigma12 + fl->sigma23 - fl->sigma13,
                     fl->sigma13 + fl->sigma23 - fl->sigma12};
    for (double l : lam)
        if (!(l > 0.0)) return fail(nullptr, TLB_EPARAM, "surface tensions give lambda_i <= 0");
    const double lamT = 3.0 / (1.0 / lam[0] + 1.0 / lam[1] + 1.0 / lam[2]);
    if (!(fl->lambda >= 0.0) || !std::isfinite(fl->lambda))
        return fail(nullptr, TLB_EPARAM, "lambda (Eq. 5) must be finite and >= 0");
    if (fl->lambda == 0.0)
        for (double l : lam)
            if (!(l > 0.5 * lamT))
                return fail(nullptr, TLB_EPARAM, "surface tensions give lambda_i <= lambda_T/2");
    if (!(fl->D > 0.0) || !(fl->M0 > 0.0)) return fail(nullptr, TLB_EPARAM, "D and M0 must be > 0");
    if (!(fl->tau1 > 0.5) || !(fl->tau2 > 0.5)) return fail(nullptr, TLB_EPARAM, "tau_i must be > 1/2");
    for (int i = 0; i < 3; ++i)
        if (!(fl->rho[i] > 0.0) || !(fl->nu[i] > 0.0))
            return fail(nullptr, TLB_EPARAM, "densities and viscosities must be > 0");
    if (!std::isfinite(fl->gravity[0]) || !std::isfinite(fl->gravity[1]) || !std::isfinite(gravity_z))
        return fail(nullptr, TLB_EPARAM, "gravity must be finite");

    tlb3_ctx* c = new tlb3_ctx();
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->prec = int(p);
    c->fl = *fl;
    c->gz = gravity_z;
    c->L = L;
    c->ws = static_cast<char*>(dev_workspace);
    c->stream = static_cast<hipStream_t>(hip_stream);
    for (int i = 0; i < 3; ++i) c->lambda[i] = lam[i];
    c->lambdaT = lamT;
    const double cs2 = 1.0 / 3.0;
    c->M[0] = fl->M0 / lam[0];
    c->M[1] = fl->M0 / lam[1];
    c->eta[0] = c->M[0] / (cs2 * (fl->tau1 - 0.5));   // Eq. 18a, one eta per component
    c->eta[1] = c->M[1] / (cs2 * (fl->tau2 - 0.5));
    fill3(c->c64, c);
    fill3(c->c32, c);
    fill_bufs(c->b64, c);
    fill_bufs(c->b32, c);
    c->grid.nx = nx;
    c->grid.ny = ny;
    c->grid.nz = nz;
    c->grid.pitch = L.pitch;
    c->grid.npad = (long long)L.npad;
    if (hipHostMalloc(reinterpret_cast<void**>(&c->health), 4 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        delete c;
        return fail(nullptr, TLB_ENOMEM, "pinned health word");
    }
    std::memset(c->health, 0, 4 * sizeof(double));
    *out = c;
    return TLB_OK;
}

tlb_status tlb3_set_geometry(tlb3_ctx* c, int px, int py, int pz, const uint8_t* material,
                             const tlb_material* mats, int n_mats, double* theta12_out) {
    if (!c || !material || n_mats < 0 || (n_mats > 0 && !mats))
        return fail(c, TLB_EINVAL, "null pointer or negative material count");
    if (n_mats > kMaxMaterials) return fail(c, TLB_EINVAL, "at most 15 materials");
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const size_t n = c->L.n;
    for (size_t i = 0; i < n; ++i)
        if (material[i] > n_mats) return fail(c, TLB_EINVAL, "material id exceeds n_mats");
    for (int m = 0; m < n_mats; ++m)
        if (mats[m].kind != TLB_WALL) return fail(c, TLB_EINVAL, "the 3-D step takes wall materials only");
    auto at = [&](int x, int y, int z) { return material[(size_t(z) * ny + y) * nx + x]; };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const bool face = (!px && (x == 0 || x == nx - 1)) || (!py && (y == 0 || y == ny - 1)) ||
                                  (!pz && (z == 0 || z == nz - 1));
                if (face && !at(x, y, z))
                    return fail(c, TLB_EINVAL, "a non-periodic direction needs wall faces");
            }
    double tab[kMatStride * (kMaxMaterials + 1)] = {};
    std::vector<double> th12(size_t(n_mats > 0 ? n_mats : 1));
    const double d2r = std::acos(-1.0) / 180.0;
    for (int m = 0; m < n_mats; ++m) {
        const double c13 = std::cos(mats[m].theta13_deg * d2r);
        const double c23 = std::cos(mats[m].theta23_deg * d2r);
        const double c12 = (c->fl.sigma13 * c13 - c->fl.sigma23 * c23) / c->fl.sigma12;  // Eq. 39
        if (!(std::fabs(c12) <= 1.0))
            return fail(c, TLB_EPARAM, "contact angles give |cos theta12| > 1 (Eq. 39)");
        if (!std::isfinite(mats[m].wall_u[0]) || !std::isfinite(mats[m].wall_u[1]))
            return fail(c, TLB_EPARAM, "wall velocity must be finite");
        double* t = &tab[kMatStride * (m + 1)];
        t[0] = c12;
        t[1] = c13;
        t[2] = c23;
        t[3] = mats[m].wall_u[0];
        t[4] = mats[m].wall_u[1];
        th12[size_t(m)] = std::acos(c12) / d2r;
    }
    std::vector<uint8_t> pad(c->L.npad, 0);
    for (size_t r = 0; r < size_t(ny) * nz; ++r)
        std::memcpy(&pad[r * c->L.pitch], material + r * nx, size_t(nx));
    hipError_t e = hipMemcpyAsync(c->ws + c->L.off_mat, pad.data(), pad.size(), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + c->L.off_mtab, tab, sizeof(tab), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "set_geometry upload");
    c->geometry = true;
    c->inited = false;
    if (theta12_out)
        for (int m = 0; m < n_mats; ++m) theta12_out[m] = th12[size_t(m)];
    return TLB_OK;
}

tlb_status tlb3_init_fields(tlb3_ctx* c, const double* c1, const double* c2, const double* ux,
                            const double* uy, const double* uz) {
    if (!c || !c1 || !c2) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->geometry) return fail(c, TLB_ESTATE, "set_geometry must precede init_fields");
    const size_t n = c->L.n;
    const double* in[5] = {c1, c2, ux, uy, uz};
    for (int f = 0; f < 5; ++f)
        if (in[f])
            for (size_t i = 0; i < n; ++i)
                if (!std::isfinite(in[f][i])) return fail(c, TLB_EINVAL, "non-finite initial field");
    double* stage = stage_ptr(c);
    hipError_t e = hipSuccess;
    for (int f = 0; f < 5 && e == hipSuccess; ++f) {
        if (in[f])
            e = hipMemcpyAsync(stage + f * n, in[f], n * sizeof(double), hipMemcpyHostToDevice,
                               c->stream);
        else
            e = hipMemsetAsync(stage + f * n, 0, n * sizeof(double), c->stream);
    }
    if (e != hipSuccess) return dev_fail(c, e, "init upload");
    e = launch3_init(c->prec, c->grid, consts_ptr(c), bufs_ptr(c), stage, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "init kernels");
    c->cur = 0;
    c->steps = 0;
    c->since_check = 0;
    c->inited = true;
    c->diverged = false;
    c->health_pending = false;
    return TLB_OK;
}

tlb_status tlb3_step(tlb3_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return fail(c, TLB_EINVAL, "null context or negative step count");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede step");
    poll_health(c);
    if (c->diverged) return fail(c, TLB_EDIVERGED, "NaN/Inf order parameter detected");
    return step_impl(c, nsteps, true);
}

tlb_status tlb3_set_check_interval(tlb3_ctx* c, int64_t interval) {
    if (!c || interval < 0) return fail(c, TLB_EINVAL, "bad interval");
    c->check_interval = interval;
    c->since_check = 0;
    return TLB_OK;
}

tlb_status tlb3_read_fields(tlb3_ctx* c, uint32_t mask, double* out) {
    if (!c || !out) return fail(c, TLB_EINVAL, "null pointer");
    if (mask == 0 || (mask & ~uint32_t(TLB3_F_ALL))) return fail(c, TLB_EINVAL, "bad field mask");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede read_fields");
    const size_t n = c->L.n;
    const size_t plane = size_t(c->nx) * c->ny;
    double* stage = stage_ptr(c);
    hipError_t e = launch3_c_mu(c->prec, c->grid, consts_ptr(c), bufs_ptr(c), c->cur, c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "readout kernels");
    // bands of z-planes whose 11 fields fit the staging area; stream order
    // keeps each band's copies ahead of the next band's kernel
    const int band = int(std::min<size_t>(size_t(c->nz), c->L.stage_doubles / (11 * plane)));
    for (int za = 0; za < c->nz && e == hipSuccess; za += band) {
        const int zb = std::min(c->nz, za + band);
        const size_t nb = size_t(zb - za) * plane;
        e = launch3_readout(c->prec, c->grid, consts_ptr(c), bufs_ptr(c), c->cur, za, zb, stage,
                            c->stream);
        int o = 0;
        for (int f = 0; f < 11 && e == hipSuccess; ++f) {
            if (!(mask & (1u << f))) continue;
            e = hipMemcpyAsync(out + size_t(o) * n + size_t(za) * plane, stage + size_t(f) * nb,
                               nb * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            ++o;
        }
    }
    if (e != hipSuccess) return dev_fail(c, e, "readout");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "readout sync");
    return TLB_OK;
}

tlb_status tlb3_read_populations(tlb3_ctx* c, double* out) {
    if (!c || !out) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede read_populations");
    const size_t n = c->L.n;
    const size_t plane = size_t(c->nx) * c->ny;
    double* stage = stage_ptr(c);
    const int band = int(std::min<size_t>(size_t(c->nz), c->L.stage_doubles / (kQ * plane)));
    hipError_t e = hipSuccess;
    for (int fam = 0; fam < 3 && e == hipSuccess; ++fam)
        for (int za = 0; za < c->nz && e == hipSuccess; za += band) {
            const int zb = std::min(c->nz, za + band);
            const size_t nb = size_t(zb - za) * plane;
            e = launch3_populations(c->prec, c->grid, bufs_ptr(c), c->cur, fam, za, zb, stage,
                                    c->stream);
            for (int k = 0; k < kQ && e == hipSuccess; ++k)
                e = hipMemcpyAsync(out + (size_t(fam) * kQ + k) * n + size_t(za) * plane,
                                   stage + size_t(k) * nb, nb * sizeof(double),
                                   hipMemcpyDeviceToHost, c->stream);
        }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "populations readout");
    return TLB_OK;
}

tlb_status tlb3_mass(tlb3_ctx* c, double out[3]) {
    if (!c || !out) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede mass");
    tlb_status st = run_mass(c);
    if (st != TLB_OK) return st;
    double r[4];
    hipError_t e = hipMemcpyAsync(r, c->ws + c->L.off_result, sizeof(r), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "mass copy");
    out[0] = r[0];
    out[1] = r[1];
    out[2] = r[2];
    if (r[3] != 0.0) {
        c->diverged = true;
        return fail(c, TLB_EDIVERGED, "NaN/Inf order parameter detected");
    }
    return TLB_OK;
}

tlb_status tlb3_time_steps(tlb3_ctx* c, int64_t nsteps, double* ms) {
    if (!c || !ms || nsteps <= 0) return fail(c, TLB_EINVAL, "bad arguments");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede time_steps");
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, c->stream);
    tlb_status st = TLB_OK;
    if (e == hipSuccess) {
        st = step_impl(c, nsteps, false);
        e = hipEventRecord(b, c->stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (st != TLB_OK) return st;
    if (e != hipSuccess) return dev_fail(c, e, "time_steps");
    *ms = double(t) / double(nsteps);
    return TLB_OK;
}

const char* tlb3_last_error(const tlb3_ctx* c) {
    return c ? c->err.c_str() : g_last_error3.c_str();
}

void tlb3_destroy(tlb3_ctx* c) {
    if (!c) return;
    // teardown: nothing to report to, so errors are dropped
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->health) (void)hipHostFree(c->health);
    delete c;
}

}  // extern "C"
