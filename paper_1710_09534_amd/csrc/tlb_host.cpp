// tlb_host.cpp -- host runtime of the C ABI declared in include/tlb.h:
// parameter derivation and validation, workspace layout, launches,
// health checks and checkpoints.  All device work goes to the context's
// stream; the only host<->device traffic is at init, readout, mass and
// checkpoint calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tlb.h"
#include "tlb_internal.h"

using namespace tlb;

namespace {

thread_local std::string g_last_error;

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    int pitch;
    size_t npad;
    size_t pop_bytes;   // one lattice (27 planes)
    size_t rest_off;    // P16: offset of the two FP32 rest planes inside a lattice
    size_t hist_bytes;
    size_t off_pop[2], off_hist[2], off_mat, off_mtab, off_desc, off_stage, off_part, off_result;
    size_t stage_doubles;
    size_t total;
};

size_t elem_bytes(int prec) { return prec == P64 ? 8 : (prec == P32 ? 4 : 2); }

Layout make_layout(int nx, int ny, int prec) {
    Layout L{};
    L.pitch = int(align_up(size_t(nx), kTileX));
    L.npad = size_t(ny) * L.pitch;
    // FP16-dev: 8 planes of (f^1_k, f^2_k) FP16 pairs and 9 FP32 g planes, then
    // the two FP32 rest planes
    size_t planes = align_up((prec == P16 ? 68 : 27 * elem_bytes(prec)) * L.npad, kAlign);
    L.rest_off = planes;
    if (prec == P16) planes += align_up(2 * L.npad * 4, kAlign);
    L.pop_bytes = planes;
    L.hist_bytes = align_up(4 * L.npad * (prec == P64 ? 8 : 4), kAlign);
    size_t o = 0;
    L.off_pop[0] = o; o += L.pop_bytes;
    L.off_pop[1] = o; o += L.pop_bytes;
    // two sets of history planes: the two-step kernel reads one and writes
    // the other (tlb_ctx::hcur names the current one)
    L.off_hist[0] = o; o += L.hist_bytes;
    L.off_hist[1] = o; o += L.hist_bytes;
    L.off_mat = o; o += align_up(L.npad, kAlign);
    L.off_mtab = o; o += align_up(kMatStride * (kMaxMaterials + 1) * sizeof(double), kAlign);
    L.off_desc = o; o += kDescBytes;
    // staging: the 4 input fields of init; readout and population copies pass
    // through it in bands of rows (at least one row of 27 planes)
    L.stage_doubles = std::max(size_t(4) * nx * ny, size_t(27) * nx);
    L.off_stage = o; o += align_up(L.stage_doubles * sizeof(double), kAlign);
    L.off_part = o; o += align_up(kReduceBlocks * 4 * sizeof(double), kAlign);
    L.off_result = o; o += kAlign;
    L.total = o;
    return L;
}

}  // namespace

struct tlb_ctx {
    int nx, ny, prec;
    tlb_fluid fl;
    Layout L;
    Grid grid;
    char* ws;
    hipStream_t stream;
    Consts<double> c64;
    Consts<float> c32;
    double lambda[3], lambdaT, M[2], eta[2];
    int px, py;
    bool geometry = false, inited = false, diverged = false;
    int64_t steps = 0;
    int64_t check_interval = 100;
    int64_t since_check = 0;
    int cur = 0;   // lattice holding the current state
    int hcur = 0;  // set of history planes holding the current history
    int pair_rows = -1;      // strip rows of the two-step kernel (0: one step per
                             // launch; -1: pair_auto_rows when the kernel applies)
    int pair_auto_rows = 0;  // default_pair_rows of this lattice
    int desc_pair_rows = 0;  // the strip rows in the uploaded device descriptor
    int n_mats = 0;
    double mtab_host[kMatStride * (kMaxMaterials + 1)] = {};
    double* health = nullptr;  // pinned host copy of the last mass result
    double* scratch = nullptr; // this GPU's static partial sums (tlb_mass_noalloc)
    alignas(16) unsigned char desc_host[kDescBytes] = {};  // last uploaded descriptor
    bool health_pending = false;
    bool rows_auto = true;      // one-step strip height never set by tlb_set_tile_rows
    std::string err;
};

namespace {

tlb_status fail(tlb_ctx* c, tlb_status s, const std::string& m) {
    if (c) c->err = m;
    g_last_error = m;
    return s;
}

tlb_status dev_fail(tlb_ctx* c, hipError_t e, const char* where) {
    return fail(c, TLB_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

PopBuf popbuf(tlb_ctx* c, int which) {
    char* base = c->ws + c->L.off_pop[which];
    PopBuf b;
    b.planes = base;
    b.rest = c->prec == P16 ? reinterpret_cast<float*>(base + c->L.rest_off) : nullptr;
    return b;
}

const void* consts_ptr(tlb_ctx* c) {
    return c->prec == P64 ? static_cast<const void*>(&c->c64) : static_cast<const void*>(&c->c32);
}

template <typename R>
void fill_consts(Consts<R>& k, const tlb_ctx* c) {
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
    k.kB = R(8.0 * f.lambda * c->lambdaT / f.D);
    k.il1 = R(1.0 / c->lambda[0]);
    k.il2 = R(1.0 / c->lambda[1]);
    k.il3 = R(1.0 / c->lambda[2]);
    for (int i = 0; i < 3; ++i) {
        k.scale[i] = 1.0f;
        k.iscale[i] = 1.0f;
    }
    k.nee = 0u;
}

// Default strip height.  W strips per CU keep a CU busiest: two in FP32 and
// FP16-dev, one in FP64.  (FP64 waves take about 245 VGPRs, so one 5-wave
// workgroup fits a CU; FP32 and FP16-dev take 128, so three fit, but a third
// strip per CU measured no faster.)  A lattice that gives every CU at least
// that many strips of 64 rows uses 64, or 128 when 128-row strips number at
// most W per CU and 64-row ones more (measured: FP64 at 1024 x 2048 and FP32
// at 2048 x 2048 run faster as one round of taller strips).
// Otherwise the height among 64 .. 8 rows with the fewest iterations per
// workgroup slot: rounds of strips over the W-per-CU slots times (groups of
// four rows + about 1.6 of prologue), the taller on a tie.  Measured on
// 64^2 .. 2048 x 1024 lattices in FP64 and FP16-dev this picks the fastest of
// 8 .. 64 rows on each (64^2 FP64: 8 rows, 14.2 against 22.1 us per step at
// 16; 512^2 FP64, whose 8-row strips would take two rounds, 16 rows; 1024^2
// FP16-dev: 32 rows, 42.8 against 49.5 us at 64).
int default_rows(int nx, int ny, int prec, int cus) {
    const int tx = (nx + kTileX - 1) / kTileX;
    auto strips = [&](int rows) { return long(tx) * ((ny + rows - 1) / rows); };
    const int slots = cus * (prec == P64 ? 1 : 2);
    if (strips(64) > slots && strips(128) <= slots) return 128;
    static const int cand[] = {64, 48, 32, 24, 16, 12, 8};
    int best = 16;
    long best_cost = -1;
    for (int rows : cand) {
        const long rounds = (strips(rows) + slots - 1) / slots;
        const long cost = rounds * (10 * std::min(rows, ny) / 4 + 16);
        if (best_cost < 0 || cost < best_cost) {
            best = rows;
            best_cost = cost;
        }
    }
    return best;
}

// Default strip height of the two-step kernel.  One 11-wave workgroup fits a
// CU, so a launch lasts about (rounds of strips per CU) x (iterations of one
// strip: a group of 4 rows each, plus 4 of pipeline); the candidate height
// with the fewest such iterations wins, the taller on a tie.  Measured on
// 64^2 .. 4096^2 FP32 lattices, this picks the fastest of 8 .. 256 rows on
// each, and every lattice is faster than at one step per launch (64^2:
// 9.9 against 14.9 us per step; 256^2: 13.4 against 21.2; 1024^2: 45.0
// against 65.5).
int default_pair_rows(int nx, int ny, int cus) {
    const long tx = (nx + kTileX - 1) / kTileX;
    static const int cand[] = {256, 128, 64, 32, 16, 8};
    int best = cand[0];
    long best_cost = -1;
    for (int rows : cand) {
        const long strips = tx * ((ny + rows - 1) / rows);
        const long rounds = (strips + cus - 1) / cus;
        const long cost = rounds * ((std::min(rows, ny) + 3) / 4 + 4);
        if (best_cost < 0 || cost < best_cost) {
            best = rows;
            best_cost = cost;
        }
    }
    return best;
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

void set_grid(tlb_ctx* c, int rows) {
    c->grid.nx = c->nx;
    c->grid.ny = c->ny;
    c->grid.pitch = c->L.pitch;
    c->grid.npad = long(c->L.npad);
    c->grid.tile_rows = rows;
    c->grid.tiles_x = (c->nx + kTileX - 1) / kTileX;   // 64-column strips
    c->grid.tiles_y = (c->ny + rows - 1) / rows;
}

// descriptor of ctx for the step kernel, with buf[cur] = current state at parity 0
template <typename R, typename H>
LatDesc<R, H> make_desc(tlb_ctx* c, const Consts<R>& k, int tile_begin, int cur, int hcur,
                        int pair_rows, int pair_tile_begin) {
    static_assert(sizeof(LatDesc<R, H>) <= kDescBytes, "descriptor slot too small");
    LatDesc<R, H> d{};
    d.g = c->grid;
    d.c = k;
    d.mat = reinterpret_cast<const uint8_t*>(c->ws + c->L.off_mat);
    d.mtab = reinterpret_cast<const double*>(c->ws + c->L.off_mtab);
    d.buf[0] = popbuf(c, 0);
    d.buf[1] = popbuf(c, 1);
    d.hist[0] = reinterpret_cast<H*>(c->ws + c->L.off_hist[0]);
    d.hist[1] = reinterpret_cast<H*>(c->ws + c->L.off_hist[1]);
    d.tile_begin = tile_begin;
    d.cur = cur;
    d.hcur = hcur;
    d.pair_rows = pair_rows;
    d.pair_tile_begin = pair_tile_begin;
    return d;
}

// writes ctx's descriptor into host buffer `out`
size_t fill_desc(tlb_ctx* c, void* out, int tile_begin, int cur, int hcur, int pair_rows = 0,
                 int pair_tile_begin = 0) {
    if (c->prec == P64) {
        auto d = make_desc<double, double>(c, c->c64, tile_begin, cur, hcur, pair_rows,
                                           pair_tile_begin);
        std::memcpy(out, &d, sizeof(d));
        return sizeof(d);
    }
    auto d = make_desc<float, float>(c, c->c32, tile_begin, cur, hcur, pair_rows, pair_tile_begin);
    std::memcpy(out, &d, sizeof(d));
    return sizeof(d);
}

// The two-step kernel serves FP32 lattices of any width (in a last strip
// narrower than 64 columns the lanes past nx step the wrapped columns that
// form the strip's right frame).
bool pair_ok(const tlb_ctx* c) { return c->prec == P32; }

// strip rows of a lone context's two-step launches (0: one step per launch)
int pair_rows_of(const tlb_ctx* c) {
    if (!pair_ok(c)) return 0;
    return c->pair_rows < 0 ? c->pair_auto_rows : c->pair_rows;
}

// Two-step strip rows of a batch member under a batch strip height h: the
// member's height rounded up to 4, at least 8 and at most h.
int member_pair_rows(int ny, int h) { return std::min(h, std::max(8, (ny + 3) / 4 * 4)); }

int pair_tiles(const tlb_ctx* c, int rows) {
    return rows > 0 ? c->grid.tiles_x * ((c->ny + rows - 1) / rows) : 0;
}

// Default batch strip height: as for a lone lattice (default_pair_rows), the
// h among 128 .. 8 rows whose launch runs the fewest strip iterations per CU,
// here rounds of all members' strips times the longest strip's row groups
// plus 4 of pipeline, the taller on a tie.  Batches of 256 x 64^2,
// 128 x 128^2 and 64 x 256^2 FP32 lattices were measured fastest at 64, 128
// and 128 rows (of 32, 64 and 128), which this picks; a batch too small to
// fill the device gets shorter strips.
int batch_pair_height(tlb_ctx* const* ctxs, int n, int cus) {
    static const int cand[] = {128, 64, 32, 16, 8};
    int best = cand[0];
    long best_cost = -1;
    for (int h : cand) {
        long strips = 0;
        int longest = 0;
        for (int i = 0; i < n; ++i) {
            const int r = member_pair_rows(ctxs[i]->ny, h);
            strips += pair_tiles(ctxs[i], r);
            longest = std::max(longest, (std::min(r, ctxs[i]->ny) + 3) / 4 + 4);
        }
        const long cost = (strips + cus - 1) / cus * longest;
        if (best_cost < 0 || cost < best_cost) {
            best = h;
            best_cost = cost;
        }
    }
    return best;
}

// One-step strip height of a batch's members whose height was never set
// (rows_auto): each takes min(h, its height rounded up to 4, at least 8), with
// h among 128 .. 8 rows giving the fewest iterations per workgroup slot over
// the whole batch (rounds of all members' strips over W slots per CU, W as in
// default_rows, times the longest strip's four-row groups plus about 1.6 of
// prologue), the taller on a tie.  Measured on batches of 64^2 and 128^2
// lattices in FP64 and FP16-dev: 256 x 64^2 FP16-dev 24.0 GLUPS at its pick of
// 32 rows against 18.1 at the lone default of 8; 32 x 64^2 FP64 7.5 GLUPS at
// 8 rows against 5.1 at 16.
int member_rows(const tlb_ctx* c, int h) {
    return c->rows_auto ? std::min(h, std::max(8, (c->ny + 3) / 4 * 4)) : c->grid.tile_rows;
}
int batch_rows(tlb_ctx* const* ctxs, int n, int prec, int cus) {
    static const int cand[] = {128, 64, 48, 32, 24, 16, 12, 8};
    const long slots = long(cus) * (prec == P64 ? 1 : 2);
    int best = cand[0];
    long best_cost = -1;
    for (int h : cand) {
        long strips = 0;
        int longest = 0;
        for (int i = 0; i < n; ++i) {
            const int r = member_rows(ctxs[i], h);
            strips += long(ctxs[i]->grid.tiles_x) * ((ctxs[i]->ny + r - 1) / r);
            longest = std::max(longest, 10 * std::min(r, ctxs[i]->ny) / 4 + 16);
        }
        const long cost = (strips + slots - 1) / slots * longest;
        if (best_cost < 0 || cost < best_cost) {
            best = h;
            best_cost = cost;
        }
    }
    return best;
}

tlb_status upload_desc(tlb_ctx* c) {
    // a lone context's launches pass cur and hcur in their parity argument
    c->desc_pair_rows = pair_rows_of(c);
    size_t n = fill_desc(c, c->desc_host, 0, 0, 0, c->desc_pair_rows, 0);
    hipError_t e = hipMemcpyAsync(c->ws + c->L.off_desc, c->desc_host, n, hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "descriptor upload");
    return TLB_OK;
}

int ntiles(const tlb_ctx* c) { return c->grid.tiles_x * c->grid.tiles_y; }

tlb_status run_mass(tlb_ctx* c, hipStream_t s) {
    hipError_t e = launch_mass(c->prec, c->grid, reinterpret_cast<uint8_t*>(c->ws + c->L.off_mat),
                               c->ws + c->L.off_hist[c->hcur],
                               reinterpret_cast<double*>(c->ws + c->L.off_part),
                               reinterpret_cast<double*>(c->ws + c->L.off_result), s);
    if (e != hipSuccess) return dev_fail(c, e, "mass reduction");
    return TLB_OK;
}

tlb_status run_mass(tlb_ctx* c) { return run_mass(c, c->stream); }

// reads the pinned copy of the last health check if it has landed
void poll_health(tlb_ctx* c) {
    if (!c->health_pending) return;
    if (hipStreamQuery(c->stream) != hipSuccess) return;  // not finished: look next time
    c->health_pending = false;
    if (c->health[3] != 0.0) c->diverged = true;
}

}  // namespace

extern "C" {

// the step kernel addresses each family of 9 planes (and the history) as one
// buffer with 32-bit offsets and discards stores at offset 2^31
static bool fits_offsets(const Layout& L, int p) {
    // FP16-dev stores g as FP32: its g family is as large as FP32's
    return 9 * L.npad * (p == TLB_FP16DEV ? 4 : elem_bytes(p)) < (size_t(1) << 31) &&
           4 * L.npad * (p == TLB_FP64 ? 8 : 4) < (size_t(1) << 31);
}

size_t tlb_workspace_bytes(int nx, int ny, tlb_precision p) {
    if (nx < 3 || ny < 3 || (p != TLB_FP64 && p != TLB_FP32 && p != TLB_FP16DEV)) return 0;
    const Layout L = make_layout(nx, ny, int(p));
    return fits_offsets(L, int(p)) ? L.total : 0;
}

tlb_status tlb_create(int nx, int ny, tlb_precision p, const tlb_fluid* fl, void* dev_workspace,
                      size_t ws_bytes, void* hip_stream, tlb_ctx** out) {
    if (!out) return fail(nullptr, TLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!fl || !dev_workspace) return fail(nullptr, TLB_EINVAL, "null fluid or workspace");
    if (nx < 3 || ny < 3) return fail(nullptr, TLB_EINVAL, "nx and ny must be >= 3");
    if (p != TLB_FP64 && p != TLB_FP32 && p != TLB_FP16DEV)
        return fail(nullptr, TLB_EINVAL, "unknown precision");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign)
        return fail(nullptr, TLB_EINVAL, "workspace not 256-byte aligned");
    Layout L = make_layout(nx, ny, int(p));
    if (!fits_offsets(L, int(p)))
        return fail(nullptr, TLB_EINVAL, "lattice too large: a family of 9 planes must stay below 2 GiB");
    if (ws_bytes < L.total) return fail(nullptr, TLB_ENOMEM, "workspace too small");
    // Eq. 7, Eq. 9
    double lam[3] = {fl->sigma12 + fl->sigma13 - fl->sigma23,
                     fl->sigma12 + fl->sigma23 - fl->sigma13,
                     fl->sigma13 + fl->sigma23 - fl->sigma12};
    for (double l : lam)
        if (!(l > 0.0)) return fail(nullptr, TLB_EPARAM, "surface tensions give lambda_i <= 0");
    double lamT = 3.0 / (1.0 / lam[0] + 1.0 / lam[1] + 1.0 / lam[2]);
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
    if (!std::isfinite(fl->gravity[0]) || !std::isfinite(fl->gravity[1]))
        return fail(nullptr, TLB_EPARAM, "gravity must be finite");

    tlb_ctx* c = new tlb_ctx();
    c->nx = nx;
    c->ny = ny;
    c->prec = int(p);
    c->fl = *fl;
    c->L = L;
    c->ws = static_cast<char*>(dev_workspace);
    c->stream = static_cast<hipStream_t>(hip_stream);
    for (int i = 0; i < 3; ++i) c->lambda[i] = lam[i];
    c->lambdaT = lamT;
    const double cs2 = 1.0 / 3.0;
    c->M[0] = fl->M0 / lam[0];                           // Eq. 12
    c->M[1] = fl->M0 / lam[1];
    c->eta[0] = c->M[0] / (cs2 * (fl->tau1 - 0.5));     // Eq. 18a per component
    c->eta[1] = c->M[1] / (cs2 * (fl->tau2 - 0.5));
    fill_consts(c->c64, c);
    fill_consts(c->c32, c);
    const int cus = device_cus();
    set_grid(c, default_rows(nx, ny, int(p), cus));
    c->pair_auto_rows = default_pair_rows(nx, ny, cus);
    if (mass_scratch(&c->scratch) != hipSuccess) {
        delete c;
        return fail(nullptr, TLB_EDEVICE, "static scratch of tlb_mass_noalloc not found on this device");
    }
    // the pinned health word of the periodic check is allocated by the first
    // check (contexts whose checks are off, such as the server's, never hold one)
    *out = c;
    return TLB_OK;
}

tlb_status tlb_set_geometry(tlb_ctx* c, int periodic_x, int periodic_y, const uint8_t* material,
                            const tlb_material* mats, int n_mats, double* theta12_out) {
    if (!c || !material || n_mats < 0 || (n_mats > 0 && !mats))
        return fail(c, TLB_EINVAL, "null pointer or negative material count");
    if (n_mats > kMaxMaterials) return fail(c, TLB_EINVAL, "at most 15 materials");
    const int nx = c->nx, ny = c->ny;
    for (long i = 0; i < long(nx) * ny; ++i)
        if (material[i] > n_mats) return fail(c, TLB_EINVAL, "material id exceeds n_mats");
    if (!periodic_x)
        for (int y = 0; y < ny; ++y)
            if (!material[long(y) * nx] || !material[long(y) * nx + nx - 1])
                return fail(c, TLB_EINVAL, "non-periodic x needs solid columns 0 and nx-1");
    if (!periodic_y)
        for (int x = 0; x < nx; ++x)
            if (!material[x] || !material[long(ny - 1) * nx + x])
                return fail(c, TLB_EINVAL, "non-periodic y needs boundary rows 0 and ny-1");
    unsigned nee = 0;
    for (int m = 0; m < n_mats; ++m) {
        if (mats[m].kind != TLB_WALL && mats[m].kind != TLB_VELOCITY)
            return fail(c, TLB_EINVAL, "unknown material kind");
        if (mats[m].kind == TLB_VELOCITY) nee |= 1u << (m + 1);
    }
    // velocity boundary nodes: rows 0 / ny-1 of a y-bounded lattice, with a
    // fluid node directly inside (the x_f of Eqs. 51-53)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int m = material[long(y) * nx + x];
            if (!((nee >> m) & 1u)) continue;
            if (periodic_y || (y != 0 && y != ny - 1))
                return fail(c, TLB_EINVAL, "velocity boundary nodes must lie in row 0 or "
                                           "ny-1 of a lattice not periodic in y");
            const int yi = y == 0 ? 1 : ny - 2;
            if (material[long(yi) * nx + x])
                return fail(c, TLB_EINVAL, "the node inside a velocity boundary node must be fluid");
        }
    double tab[kMatStride * (kMaxMaterials + 1)] = {};
    std::vector<double> th12(size_t(n_mats > 0 ? n_mats : 1));
    const double d2r = std::acos(-1.0) / 180.0;
    for (int m = 0; m < n_mats; ++m) {
        if (!std::isfinite(mats[m].wall_u[0]) || !std::isfinite(mats[m].wall_u[1]))
            return fail(c, TLB_EPARAM, "wall velocity must be finite");
        double* t = &tab[kMatStride * (m + 1)];
        t[3] = mats[m].wall_u[0];
        t[4] = mats[m].wall_u[1];
        if (mats[m].kind == TLB_VELOCITY) {
            th12[size_t(m)] = std::nan("");
            continue;
        }
        double c13 = std::cos(mats[m].theta13_deg * d2r);
        double c23 = std::cos(mats[m].theta23_deg * d2r);
        double c12 = (c->fl.sigma13 * c13 - c->fl.sigma23 * c23) / c->fl.sigma12;  // Eq. 39
        if (!(std::fabs(c12) <= 1.0))
            return fail(c, TLB_EPARAM, "contact angles give |cos theta12| > 1 (Eq. 39)");
        t[0] = c12;
        t[1] = c13;
        t[2] = c23;
        th12[size_t(m)] = std::acos(c12) / d2r;
    }
    // upload the padded material plane
    std::vector<uint8_t> pad(c->L.npad, 0);
    for (int y = 0; y < ny; ++y) std::memcpy(&pad[size_t(y) * c->L.pitch], material + long(y) * nx, size_t(nx));
    hipError_t e = hipMemcpyAsync(c->ws + c->L.off_mat, pad.data(), pad.size(), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + c->L.off_mtab, tab, sizeof(tab), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "set_geometry upload");
    std::memcpy(c->mtab_host, tab, sizeof(tab));
    c->c64.nee = nee;
    c->c32.nee = nee;
    c->n_mats = n_mats;
    c->px = periodic_x != 0;
    c->py = periodic_y != 0;
    c->geometry = true;
    c->inited = false;
    if (theta12_out)
        for (int m = 0; m < n_mats; ++m) theta12_out[m] = th12[size_t(m)];
    return TLB_OK;
}

tlb_status tlb_init_fields(tlb_ctx* c, const double* c1, const double* c2, const double* ux,
                           const double* uy) {
    if (!c || !c1 || !c2) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->geometry) return fail(c, TLB_ESTATE, "set_geometry must precede init_fields");
    const size_t n = size_t(c->nx) * c->ny;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(c1[i]) || !std::isfinite(c2[i]) || (ux && !std::isfinite(ux[i])) ||
            (uy && !std::isfinite(uy[i])))
            return fail(c, TLB_EINVAL, "non-finite initial field");
    std::vector<double> host(4 * n, 0.0);
    std::memcpy(host.data(), c1, n * sizeof(double));
    std::memcpy(host.data() + n, c2, n * sizeof(double));
    if (ux) std::memcpy(host.data() + 2 * n, ux, n * sizeof(double));
    if (uy) std::memcpy(host.data() + 3 * n, uy, n * sizeof(double));
    // FP16 storage scale of the two order-parameter families: a power of two
    // that maps the largest initial moving population (bounded by the
    // velocity and mu ranges) well inside the FP16 range, with 2^6 headroom
    // for transients.  The g family is stored as FP32 (scale 1).
    if (c->prec == P16) {
        double umax = 0.0;
        for (size_t i = 0; i < n; ++i) {
            double u2 = (ux ? ux[i] * ux[i] : 0.0) + (uy ? uy[i] * uy[i] : 0.0);
            umax = std::fmax(umax, std::sqrt(u2));
        }
        for (int m = 1; m <= c->n_mats; ++m)   // walls and velocity boundaries drive the flow
            umax = std::fmax(umax, std::hypot(c->mtab_host[kMatStride * m + 3],
                                              c->mtab_host[kMatStride * m + 4]));
        const double m = std::fmax(umax, 0.02);
        const double fmaxv[2] = {m + 1e-2, m + 1e-2};
        for (int f = 0; f < 2; ++f) {
            int ex = int(std::floor(std::log2(1024.0 / fmaxv[f])));
            c->c32.scale[f] = std::ldexp(1.0f, ex);
            c->c32.iscale[f] = std::ldexp(1.0f, -ex);
        }
    }
    double* stage = reinterpret_cast<double*>(c->ws + c->L.off_stage);
    hipError_t e = hipMemcpyAsync(stage, host.data(), 4 * n * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "init upload");
    Grid g = c->grid;
    e = launch_init(c->prec, g, consts_ptr(c), reinterpret_cast<uint8_t*>(c->ws + c->L.off_mat),
                    reinterpret_cast<double*>(c->ws + c->L.off_mtab), stage, popbuf(c, 0),
                    c->ws + c->L.off_hist[0], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "init kernel");
    c->cur = 0;
    c->hcur = 0;
    c->steps = 0;
    c->since_check = 0;
    c->inited = true;
    c->diverged = false;
    c->health_pending = false;
    return upload_desc(c);
}

// optional step-kernel parts this lattice needs (launch_step's features)
static unsigned features(const tlb_ctx* c) {
    return (c->c64.nee != 0u ? 1u : 0u) | (c->fl.lambda != 0.0 ? 2u : 0u);
}

static tlb_status step_impl(tlb_ctx* c, int64_t nsteps, bool checks) {
    for (int64_t s = 0; s < nsteps;) {
        // two steps in one launch when the kernel applies and no health check
        // falls between them
        const bool room = !checks || c->check_interval <= 0 ||
                          c->check_interval - c->since_check >= 2;
        const int pr = pair_rows_of(c);
        if (pr != c->desc_pair_rows) {   // the descriptor must carry the strip height
            tlb_status st = upload_desc(c);
            if (st != TLB_OK) return st;
        }
        const int n = (pr > 0 && nsteps - s >= 2 && room) ? 2 : 1;
        hipError_t e;
        const int parity = c->cur | (c->hcur << 1);
        if (n == 2) {
            e = launch_step2(c->prec, features(c), c->ws + c->L.off_desc, 1, pair_tiles(c, pr),
                             parity, c->stream);
        } else {
            e = launch_step(c->prec, features(c), c->ws + c->L.off_desc, 1, ntiles(c), parity,
                            c->stream);
        }
        if (e != hipSuccess) return dev_fail(c, e, "step kernel");
        c->cur = 1 - c->cur;
        if (n == 2) c->hcur = 1 - c->hcur;   // the two-step kernel wrote the other set
        c->steps += n;
        s += n;
        if (checks && c->check_interval > 0 && (c->since_check += n) >= c->check_interval) {
            c->since_check = 0;
            if (!c->health) {
                if (hipHostMalloc(reinterpret_cast<void**>(&c->health), 4 * sizeof(double)) !=
                    hipSuccess)
                    return fail(c, TLB_ENOMEM, "pinned health word");
                std::memset(c->health, 0, 4 * sizeof(double));
            }
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

tlb_status tlb_step(tlb_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return fail(c, TLB_EINVAL, "null context or negative step count");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede step");
    poll_health(c);
    if (c->diverged) return fail(c, TLB_EDIVERGED, "NaN/Inf order parameter detected");
    return step_impl(c, nsteps, true);
}

tlb_status tlb_set_check_interval(tlb_ctx* c, int64_t interval) {
    if (!c || interval < 0) return fail(c, TLB_EINVAL, "bad interval");
    c->check_interval = interval;
    c->since_check = 0;
    return TLB_OK;
}

int64_t tlb_step_count(const tlb_ctx* c) { return c ? c->steps : -1; }

tlb_status tlb_set_tile_rows(tlb_ctx* c, int rows) {
    if (!c || rows < 8 || rows > 4096 || rows % 4)
        return fail(c, TLB_EINVAL, "strip rows must be a multiple of 4 in [8, 4096]");
    set_grid(c, rows);
    c->rows_auto = false;
    return c->inited ? upload_desc(c) : TLB_OK;
}

tlb_status tlb_set_pair_rows(tlb_ctx* c, int rows) {
    if (!c) return fail(c, TLB_EINVAL, "null context");
    if (rows != -1 && rows != 0) {
        if (rows < 8 || rows > 4096 || rows % 4)
            return fail(c, TLB_EINVAL,
                        "pair strip rows must be 0, -1 or a multiple of 4 in [8, 4096]");
        if (!pair_ok(c))
            return fail(c, TLB_EINVAL, "the two-step kernel needs FP32 storage");
    }
    c->pair_rows = rows;
    // the device descriptor carries the strip height
    return c->inited ? upload_desc(c) : TLB_OK;
}

tlb_status tlb_read_fields(tlb_ctx* c, uint32_t mask, double* out) {
    if (!c || !out) return fail(c, TLB_EINVAL, "null pointer");
    if (mask == 0 || (mask & ~uint32_t(TLB_F_ALL))) return fail(c, TLB_EINVAL, "bad field mask");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede read_fields");
    const size_t n = size_t(c->nx) * c->ny;
    double* stage = reinterpret_cast<double*>(c->ws + c->L.off_stage);
    // bands of rows whose 10 fields fit the staging area; stream order keeps
    // each band's copies ahead of the next band's kernel
    const int band = int(std::min<size_t>(size_t(c->ny), c->L.stage_doubles / (10 * size_t(c->nx))));
    hipError_t e = hipSuccess;
    for (int ya = 0; ya < c->ny && e == hipSuccess; ya += band) {
        const int yb = std::min(c->ny, ya + band);
        const size_t nb = size_t(yb - ya) * c->nx;
        e = launch_readout(c->prec, c->grid, consts_ptr(c),
                           reinterpret_cast<uint8_t*>(c->ws + c->L.off_mat),
                           reinterpret_cast<double*>(c->ws + c->L.off_mtab), popbuf(c, c->cur), ya,
                           yb, stage, c->stream);
        if (e != hipSuccess) return dev_fail(c, e, "readout kernel");
        int o = 0;
        for (int f = 0; f < 10 && e == hipSuccess; ++f) {
            if (!(mask & (1u << f))) continue;
            e = hipMemcpyAsync(out + size_t(o) * n + size_t(ya) * c->nx, stage + size_t(f) * nb,
                               nb * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            ++o;
        }
    }
    if (e != hipSuccess) return dev_fail(c, e, "readout copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "readout sync");
    return TLB_OK;
}

tlb_status tlb_read_populations(tlb_ctx* c, double* out) {
    if (!c || !out) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede read_populations");
    const size_t n = size_t(c->nx) * c->ny;
    double* stage = reinterpret_cast<double*>(c->ws + c->L.off_stage);
    const int band = int(std::min<size_t>(size_t(c->ny), c->L.stage_doubles / (27 * size_t(c->nx))));
    hipError_t e = hipSuccess;
    for (int ya = 0; ya < c->ny && e == hipSuccess; ya += band) {
        const int yb = std::min(c->ny, ya + band);
        const size_t nb = size_t(yb - ya) * c->nx;
        e = launch_populations(c->prec, c->grid, consts_ptr(c),
                               reinterpret_cast<uint8_t*>(c->ws + c->L.off_mat), popbuf(c, c->cur),
                               ya, yb, stage, c->stream);
        for (int q = 0; q < 27 && e == hipSuccess; ++q)
            e = hipMemcpyAsync(out + size_t(q) * n + size_t(ya) * c->nx, stage + size_t(q) * nb,
                               nb * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "read_populations");
    return TLB_OK;
}

tlb_status tlb_mass(tlb_ctx* c, double out[3]) {
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

extern "C++" {
namespace tlb {
int health_enqueue(tlb_ctx* c, hipStream_t s, double* host4) {
    if (!c || !host4 || !c->inited) return TLB_EINVAL;
    tlb_status st = run_mass(c, s);
    if (st != TLB_OK) return st;
    hipError_t e = hipMemcpyAsync(host4, c->ws + c->L.off_result, 4 * sizeof(double),
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return dev_fail(c, e, "health copy");
    return TLB_OK;
}
}  // namespace tlb
}  // extern "C++"

tlb_status tlb_mass_noalloc(tlb_ctx* c, double* dev_out) {
    static_assert(kScratchDoubles >= kReduceBlocks * 4, "static scratch holds every partial sum");
    if (!c || !dev_out) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede mass");
    if (!c->scratch) return fail(c, TLB_EDEVICE, "static scratch not resolved");
    hipError_t e = launch_mass(c->prec, c->grid, reinterpret_cast<uint8_t*>(c->ws + c->L.off_mat),
                               c->ws + c->L.off_hist[c->hcur], c->scratch, dev_out, c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "mass reduction");
    return TLB_OK;
}

tlb_status tlb_checkpoint_bytes(const tlb_ctx* c, size_t* bytes) {
    if (!c || !bytes) {
        g_last_error = "null pointer";
        return TLB_EINVAL;
    }
    *bytes = 64 + c->L.pop_bytes + c->L.hist_bytes;
    return TLB_OK;
}

tlb_status tlb_checkpoint_save(tlb_ctx* c, void* buf) {
    if (!c || !buf) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->inited) return fail(c, TLB_ESTATE, "nothing to save before init_fields");
    char* b = static_cast<char*>(buf);
    std::memset(b, 0, 64);
    std::memcpy(b, "TLBCKPT1", 8);
    int32_t hdr[4] = {c->nx, c->ny, c->prec, 0};
    std::memcpy(b + 8, hdr, sizeof(hdr));
    std::memcpy(b + 24, &c->steps, 8);
    std::memcpy(b + 32, c->c32.scale, 3 * sizeof(float));
    std::memcpy(b + 44, c->c32.iscale, 3 * sizeof(float));
    hipError_t e = hipMemcpyAsync(b + 64, c->ws + c->L.off_pop[c->cur], c->L.pop_bytes,
                                  hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b + 64 + c->L.pop_bytes, c->ws + c->L.off_hist[c->hcur], c->L.hist_bytes,
                           hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "checkpoint save");
    return TLB_OK;
}

tlb_status tlb_checkpoint_load(tlb_ctx* c, const void* buf) {
    if (!c || !buf) return fail(c, TLB_EINVAL, "null pointer");
    if (!c->geometry) return fail(c, TLB_ESTATE, "set_geometry must precede checkpoint_load");
    const char* b = static_cast<const char*>(buf);
    int32_t hdr[4];
    std::memcpy(hdr, b + 8, sizeof(hdr));
    if (std::memcmp(b, "TLBCKPT1", 8) || hdr[0] != c->nx || hdr[1] != c->ny || hdr[2] != c->prec)
        return fail(c, TLB_EINVAL, "checkpoint does not match this context");
    int64_t steps;
    std::memcpy(&steps, b + 24, 8);
    hipError_t e = hipMemcpyAsync(c->ws + c->L.off_pop[0], b + 64, c->L.pop_bytes,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + c->L.off_hist[0], b + 64 + c->L.pop_bytes, c->L.hist_bytes,
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return dev_fail(c, e, "checkpoint load");
    std::memcpy(c->c32.scale, b + 32, 3 * sizeof(float));
    std::memcpy(c->c32.iscale, b + 44, 3 * sizeof(float));
    c->cur = 0;
    c->hcur = 0;
    c->steps = steps;
    c->since_check = 0;
    c->inited = true;
    c->diverged = false;
    c->health_pending = false;
    return upload_desc(c);
}

tlb_status tlb_time_steps(tlb_ctx* c, int64_t nsteps, double* ms) {
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

// ------------------------------------------------------------------ batches
}  // extern "C"

struct tlb_batch {
    char* dev;            // caller-owned device table (kDescBytes per lattice)
    size_t bytes;
    int cap;
    hipStream_t stream;
    int prec = -1;
    std::vector<tlb_ctx*> ctxs;
    std::vector<int> base_cur;         // each member's cur when the table was written
    std::vector<int> base_hcur;        // and its hcur (batch steps keep it)
    std::vector<unsigned char> host;   // staged table
    int total_tiles = 0;
    unsigned features = 0;             // union of the members' step-kernel features
    int parity = 0;                    // parity of the next step relative to the table
    int pair_rows = -1;                // two-step strip rows requested (0: one step per launch,
                                       // -1: member_pair_rows under batch_pair_height)
    bool pairs = false;                // pair_rows > 0 and every member can take two steps
    int pair_total_tiles = 0;          // sum of the members' two-step strips
    int hparity = 0;                   // history set of the next launch relative to the table
    std::vector<std::pair<int, int>> tuned_pair_rows;  // (member height, two-step strip rows)
                                       // from tlb_batch_autotune_pair_rows, used while pair_rows == -1
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_steps = 0;
    std::string err;
};

namespace {
tlb_status bfail(tlb_batch* b, tlb_status s, const std::string& m) {
    if (b) b->err = m;
    g_last_error = m;
    return s;
}
void drop_graph(tlb_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = 0;
}
}  // namespace

extern "C" {

size_t tlb_batch_table_bytes(int max_lattices) {
    return max_lattices > 0 ? size_t(max_lattices) * kDescBytes : 0;
}

tlb_status tlb_batch_create(int max_lattices, void* dev_table, size_t bytes, void* hip_stream,
                            tlb_batch** out) {
    if (!out) return bfail(nullptr, TLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_lattices <= 0 || !dev_table || bytes < tlb_batch_table_bytes(max_lattices))
        return bfail(nullptr, TLB_EINVAL, "bad batch capacity or table");
    if (reinterpret_cast<uintptr_t>(dev_table) % kAlign)
        return bfail(nullptr, TLB_EINVAL, "table not 256-byte aligned");
    tlb_batch* b = new tlb_batch();
    b->dev = static_cast<char*>(dev_table);
    b->bytes = bytes;
    b->cap = max_lattices;
    b->stream = static_cast<hipStream_t>(hip_stream);
    *out = b;
    return TLB_OK;
}

tlb_status tlb_batch_set(tlb_batch* b, tlb_ctx* const* ctxs, int n) {
    if (!b || (n > 0 && !ctxs) || n < 0) return bfail(b, TLB_EINVAL, "null batch or contexts");
    if (n > b->cap) return bfail(b, TLB_EINVAL, "more lattices than the batch capacity");
    int prec = -1, tiles = 0;
    unsigned feat = 0;
    for (int i = 0; i < n; ++i) {
        tlb_ctx* c = ctxs[i];
        if (!c) return bfail(b, TLB_EINVAL, "null context in batch");
        feat |= features(c);
        if (!c->inited) return bfail(b, TLB_ESTATE, "every context must be initialised");
        if (c->diverged) return bfail(b, TLB_EDIVERGED, "a context has diverged");
        if (prec >= 0 && c->prec != prec) return bfail(b, TLB_EINVAL, "mixed precisions in batch");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return bfail(b, TLB_EINVAL, "context listed twice");
        prec = c->prec;
        tiles += ntiles(c);
    }
    // finish pending work of the contexts on their own streams first
    for (int i = 0; i < n; ++i)
        if (hipStreamSynchronize(ctxs[i]->stream) != hipSuccess)
            return bfail(b, TLB_EDEVICE, "context stream sync failed");
    // members whose one-step strip height was never set take the batch's
    // (batch_rows); their own descriptor follows, so that stepping one alone
    // stays consistent (results do not depend on strip heights)
    bool any_auto = false;
    for (int i = 0; i < n; ++i) any_auto = any_auto || ctxs[i]->rows_auto;
    if (any_auto) {
        const int h1 = batch_rows(ctxs, n, prec, device_cus());
        tiles = 0;
        for (int i = 0; i < n; ++i) {
            tlb_ctx* c = ctxs[i];
            const int r = member_rows(c, h1);
            if (r != c->grid.tile_rows) {
                set_grid(c, r);
                const tlb_status st = upload_desc(c);
                if (st != TLB_OK) return bfail(b, st, "member descriptor: " + c->err);
            }
            tiles += ntiles(c);
        }
    }
    b->host.assign(size_t(n > 0 ? n : 1) * kDescBytes, 0);
    bool pairs = b->pair_rows != 0 && n > 0;
    for (int i = 0; i < n; ++i) pairs = pairs && pair_ok(ctxs[i]);
    const int h = pairs && b->pair_rows < 0 ? batch_pair_height(ctxs, n, device_cus()) : 0;
    int begin = 0, pbegin = 0;
    for (int i = 0; i < n; ++i) {
        int pr = !pairs ? 0 : (b->pair_rows > 0 ? b->pair_rows : member_pair_rows(ctxs[i]->ny, h));
        if (pairs && b->pair_rows < 0)
            for (const auto& t : b->tuned_pair_rows)
                if (t.first == ctxs[i]->ny) pr = t.second;
        fill_desc(ctxs[i], b->host.data() + size_t(i) * kDescBytes, begin, ctxs[i]->cur,
                  ctxs[i]->hcur, pr, pbegin);
        begin += ntiles(ctxs[i]);
        pbegin += pair_tiles(ctxs[i], pr);
    }
    b->pairs = pairs;
    b->pair_total_tiles = pbegin;
    if (n > 0) {
        hipError_t e = hipMemcpyAsync(b->dev, b->host.data(), size_t(n) * kDescBytes,
                                      hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return bfail(b, TLB_EDEVICE, std::string("batch table upload: ") + hipGetErrorString(e));
    }
    drop_graph(b);
    b->ctxs.assign(ctxs, ctxs + n);
    b->base_cur.resize(size_t(n));
    b->base_hcur.resize(size_t(n));
    for (int i = 0; i < n; ++i) {
        b->base_cur[size_t(i)] = ctxs[i]->cur;
        b->base_hcur[size_t(i)] = ctxs[i]->hcur;
    }
    b->prec = prec;
    b->total_tiles = tiles;
    b->features = feat;
    b->parity = 0;
    b->hparity = 0;
    return TLB_OK;
}

tlb_status tlb_batch_set_pair_rows(tlb_batch* b, int rows) {
    if (!b) return bfail(b, TLB_EINVAL, "null batch");
    if (rows != 0 && rows != -1 && (rows < 8 || rows > 4096 || rows % 4))
        return bfail(b, TLB_EINVAL,
                     "pair strip rows must be 0, -1 or a multiple of 4 in [8, 4096]");
    b->pair_rows = rows;
    b->tuned_pair_rows.clear();
    if (b->ctxs.empty()) return TLB_OK;
    // re-register the members: the table carries the strip layout
    const std::vector<tlb_ctx*> members = b->ctxs;
    for (size_t i = 0; i < members.size(); ++i)
        if (((b->base_cur[i] + b->parity) & 1) != members[i]->cur ||
            (b->base_hcur[i] ^ b->hparity) != members[i]->hcur)
            return bfail(b, TLB_ESTATE, "a member was stepped outside the batch: call tlb_batch_set");
    if (hipStreamSynchronize(b->stream) != hipSuccess)
        return bfail(b, TLB_EDEVICE, "batch stream sync failed");
    return tlb_batch_set(b, members.data(), int(members.size()));
}

// records `steps` (even) step launches starting at parity 0 into a graph
tlb_status tlb_batch_use_graph(tlb_batch* b, int steps) {
    if (!b || steps < 0 || (steps & 1)) return bfail(b, TLB_EINVAL, "graph steps must be even and >= 0");
    if (b->pairs && (steps & 3))
        return bfail(b, TLB_EINVAL, "with two steps per launch, graph steps must be a multiple of 4");
    drop_graph(b);
    if (steps == 0 || b->ctxs.empty()) return TLB_OK;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, TLB_EDEVICE, std::string("begin capture: ") + hipGetErrorString(e));
    hipError_t le = hipSuccess;
    if (b->pairs) {
        // two steps per launch: steps / 2 launches, each turning over the
        // population buffer and the history set
        for (int s = 0; s < steps / 2 && le == hipSuccess; ++s)
            le = launch_step2(b->prec, b->features, b->dev, int(b->ctxs.size()),
                              b->pair_total_tiles, (s & 1) | ((s & 1) << 1), b->stream);
    } else {
        for (int s = 0; s < steps && le == hipSuccess; ++s)
            le = launch_step(b->prec, b->features, b->dev, int(b->ctxs.size()), b->total_tiles,
                             s & 1, b->stream);
    }
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (le != hipSuccess || e != hipSuccess) {
        drop_graph(b);
        return bfail(b, TLB_EDEVICE, "graph capture failed");
    }
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return bfail(b, TLB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    b->graph_steps = steps;
    return TLB_OK;
}

tlb_status tlb_batch_step(tlb_batch* b, int64_t nsteps) {
    if (!b || nsteps < 0) return bfail(b, TLB_EINVAL, "null batch or negative steps");
    if (b->ctxs.empty() || nsteps == 0) return TLB_OK;
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
        const tlb_ctx* c = b->ctxs[i];
        if (c->diverged) return bfail(b, TLB_EDIVERGED, "a context has diverged");
        if (((b->base_cur[i] + b->parity) & 1) != c->cur || (b->base_hcur[i] ^ b->hparity) != c->hcur)
            return bfail(b, TLB_ESTATE, "a member was stepped outside the batch: call tlb_batch_set");
    }
    int64_t done = 0;
    int launches = 0, pair_launches = 0;   // beyond the graph replays (which change neither)
    const int nd = int(b->ctxs.size());
    // the members take the launches that went out, also when a later one fails
    auto settle = [&]() {
        for (tlb_ctx* c : b->ctxs) {
            c->cur ^= launches & 1;
            c->hcur ^= pair_launches & 1;
            c->steps += done;
        }
    };
    while (done < nsteps) {
        hipError_t e;
        if (b->exec && b->parity == 0 && b->hparity == 0 && nsteps - done >= b->graph_steps) {
            e = hipGraphLaunch(b->exec, b->stream);
            if (e != hipSuccess) {
                settle();
                return bfail(b, TLB_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
            }
            done += b->graph_steps;
            continue;   // an even number of launches: parity and history set unchanged
        }
        const int parity = b->parity | (b->hparity << 1);
        const bool pair = b->pairs && nsteps - done >= 2;
        if (pair)
            e = launch_step2(b->prec, b->features, b->dev, nd, b->pair_total_tiles, parity,
                             b->stream);
        else
            e = launch_step(b->prec, b->features, b->dev, nd, b->total_tiles, parity, b->stream);
        if (e != hipSuccess) {
            settle();
            return bfail(b, TLB_EDEVICE, std::string("batch step: ") + hipGetErrorString(e));
        }
        if (pair) {
            b->hparity ^= 1;   // the two-step kernel wrote the other history set
            ++pair_launches;
        }
        done += pair ? 2 : 1;
        b->parity ^= 1;
        ++launches;
    }
    settle();
    return TLB_OK;
}

tlb_status tlb_batch_sync(tlb_batch* b) {
    if (!b) return bfail(b, TLB_EINVAL, "null batch");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, TLB_EDEVICE, std::string("batch sync: ") + hipGetErrorString(e));
    return TLB_OK;
}

namespace {
// mean time per step of `steps` batched steps, HIP events on the batch stream
tlb_status time_batch_steps(tlb_batch* b, int steps, double* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    tlb_status st = e == hipSuccess ? tlb_batch_step(b, steps) : TLB_EDEVICE;
    if (st == TLB_OK) {
        e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        *ms = double(f) / steps;
        if (e != hipSuccess) st = TLB_EDEVICE;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st == TLB_EDEVICE) return bfail(b, st, "autotune timing");
    return st;
}
}  // namespace

tlb_status tlb_batch_autotune_rows(tlb_batch* b, int steps_per_candidate, int* best_rows) {
    if (!b || steps_per_candidate <= 0) return bfail(b, TLB_EINVAL, "bad arguments");
    if (b->ctxs.empty()) return bfail(b, TLB_ESTATE, "tlb_batch_set must precede autotune");
    static const int cand[] = {16, 24, 32, 48, 64, 96, 128};
    const std::vector<tlb_ctx*> members = b->ctxs;
    // the candidates are strip heights of the one-step kernel: time it alone
    // (the final registration restores two steps per launch)
    const int pair_rows = b->pair_rows;
    b->pair_rows = 0;
    struct Restore {
        tlb_batch* b;
        int rows;
        ~Restore() { b->pair_rows = rows; }
    } restore{b, pair_rows};
    // size classes: members of the same height share a strip height
    std::vector<int> heights;
    for (tlb_ctx* c : members)
        if (std::find(heights.begin(), heights.end(), c->ny) == heights.end())
            heights.push_back(c->ny);
    std::sort(heights.begin(), heights.end(), std::greater<int>());
    std::vector<int> rows(heights.size());
    for (size_t h = 0; h < heights.size(); ++h) {
        rows[h] = members[0]->grid.tile_rows;
        for (tlb_ctx* c : members)
            if (c->ny == heights[h]) rows[h] = c->grid.tile_rows;
    }
    auto apply = [&]() -> tlb_status {
        for (tlb_ctx* c : members) {
            const size_t h = size_t(std::find(heights.begin(), heights.end(), c->ny) - heights.begin());
            tlb_status st = tlb_set_tile_rows(c, rows[h]);
            if (st != TLB_OK) return bfail(b, st, std::string("set rows: ") + c->err);
        }
        return tlb_batch_set(b, members.data(), int(members.size()));
    };
    auto time_batch = [&](double* ms) { return time_batch_steps(b, steps_per_candidate, ms); };
    // one pass of coordinate descent over the size classes, tallest first:
    // every member of a class takes the candidate that gives the shortest
    // batched step with the other classes at their current strip heights
    for (size_t h = 0; h < heights.size(); ++h) {
        const int limit = std::max(16, (heights[h] + 3) / 4 * 4);
        int best = rows[h];
        double best_ms = 1e30;
        for (int r : cand) {
            if (r > limit) break;
            rows[h] = r;
            tlb_status st = apply();
            double ms = 0.0;
            if (st == TLB_OK) st = time_batch(&ms);
            if (st != TLB_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best = r;
            }
        }
        rows[h] = best;
    }
    b->pair_rows = pair_rows;
    tlb_status st = apply();
    if (st != TLB_OK) return st;
    if (best_rows) *best_rows = rows.empty() ? 0 : rows[0];
    return TLB_OK;
}

tlb_status tlb_batch_autotune_pair_rows(tlb_batch* b, int steps_per_candidate, int* best_rows) {
    if (!b || steps_per_candidate <= 0) return bfail(b, TLB_EINVAL, "bad arguments");
    if (b->ctxs.empty()) return bfail(b, TLB_ESTATE, "tlb_batch_set must precede autotune");
    if (!b->pairs || b->pair_rows >= 0)
        return bfail(b, TLB_ESTATE, "the batch does not take two steps per launch at default heights");
    static const int cand[] = {8, 16, 32, 64, 128};
    const std::vector<tlb_ctx*> members = b->ctxs;
    const int steps = (steps_per_candidate + 1) / 2 * 2;   // whole two-step launches
    // size classes, tallest first, starting from the heights the batch runs now
    std::vector<std::pair<int, int>> cls;
    for (tlb_ctx* c : members) {
        bool seen = false;
        for (const auto& t : cls) seen = seen || t.first == c->ny;
        if (!seen) cls.push_back({c->ny, 0});
    }
    std::sort(cls.begin(), cls.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& z) {
        return a.first > z.first;
    });
    const int h0 = batch_pair_height(members.data(), int(members.size()), device_cus());
    for (auto& t : cls) {
        t.second = member_pair_rows(t.first, h0);
        for (const auto& u : b->tuned_pair_rows)
            if (u.first == t.first) t.second = u.second;
    }
    // one pass of coordinate descent over the classes: every member of a class
    // takes the candidate that gives the shortest batched step with the other
    // classes at their current heights (candidates stop at the first one that
    // covers the whole lattice in one strip row)
    for (size_t h = 0; h < cls.size(); ++h) {
        int best = cls[h].second;
        double best_ms = 1e30;
        for (int r : cand) {
            cls[h].second = r;
            b->tuned_pair_rows = cls;
            tlb_status st = tlb_batch_set(b, members.data(), int(members.size()));
            double ms = 0.0;
            if (st == TLB_OK) st = time_batch_steps(b, steps, &ms);
            if (st != TLB_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best = r;
            }
            if (r >= cls[h].first) break;
        }
        cls[h].second = best;
    }
    b->tuned_pair_rows = cls;
    tlb_status st = tlb_batch_set(b, members.data(), int(members.size()));
    if (st == TLB_OK && best_rows) *best_rows = cls[0].second;
    return st;
}

const char* tlb_batch_last_error(const tlb_batch* b) {
    return b ? b->err.c_str() : g_last_error.c_str();
}

void tlb_batch_destroy(tlb_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    delete b;
}

// ---------------------------------------------------------------- autotuner
tlb_status tlb_autotune_rows(tlb_ctx* c, int steps_per_candidate, int* best_rows) {
    if (!c || steps_per_candidate <= 0) return fail(c, TLB_EINVAL, "bad arguments");
    if (!c->inited) return fail(c, TLB_ESTATE, "init_fields must precede autotune");
    static const int cand[] = {16, 24, 32, 48, 64, 96, 128};
    // the candidates are strip heights of the one-step kernel: time it alone,
    // then restore the two-step setting (and the descriptor that carries it)
    const int pair_rows = c->pair_rows;
    c->pair_rows = 0;
    int best = c->grid.tile_rows;
    double best_ms = 1e30;
    const int limit = ((c->ny + 3) / 4) * 4;
    tlb_status st = TLB_OK;
    for (int rows : cand) {
        if (rows > (limit < 16 ? 16 : limit)) break;
        st = tlb_set_tile_rows(c, rows);
        double ms = 0.0;
        if (st == TLB_OK) st = tlb_time_steps(c, steps_per_candidate, &ms);
        if (st != TLB_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = rows;
        }
    }
    c->pair_rows = pair_rows;
    tlb_status st2 = tlb_set_tile_rows(c, st == TLB_OK ? best : c->grid.tile_rows);
    if (st != TLB_OK) return st;
    if (st2 != TLB_OK) return st2;
    if (best_rows) *best_rows = best;
    return TLB_OK;
}

const char* tlb_last_error(const tlb_ctx* c) {
    if (c) return c->err.c_str();
    return g_last_error.c_str();
}

void tlb_destroy(tlb_ctx* c) {
    if (!c) return;
    // teardown: nothing to report to, so errors are dropped
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->health) (void)hipHostFree(c->health);
    delete c;
}

}  // extern "C"
