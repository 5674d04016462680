// tlb_probe.hip -- streaming references for the bandwidth figures reported
// beside the step kernel.  Not part of the method: they move bytes the way
// the step kernel does, without its arithmetic, so that the fraction of HBM
// peak the step reaches can be read against what this device sustains for
// the same access pattern.
//   kind 0: copy of 16-byte words (dwordx4 loads and stores), grid-stride
//           over the buffer, non-temporal stores;
//   kind 1: the step kernel's access shape: workgroups of four row waves,
//           one lane per column of a 64-column strip of tile_rows rows, each
//           node reads 31 FP32 planes (27 population planes at x - e_k of the
//           D2Q9 directions, wrapped periodically, and 4 history planes at x)
//           and writes 31 planes at x with non-temporal stores.
#include <hip/hip_runtime.h>

#include "../../include/tlb.h"
#include "tlb_internal.h"

namespace tlb {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int PEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int PEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// grid-stride copy, one 16-byte word per lane and iteration, non-temporal
// stores; the grid is four 256-thread blocks per compute unit (of the
// variants timed on this device -- one or four words per iteration,
// non-temporal loads and/or stores, 1024 to 16384 blocks -- the fastest:
// 5.8 TB/s read plus write on 1 GiB)
__global__ __launch_bounds__(256) void copy16_kernel(const f4* __restrict__ src,
                                                     f4* __restrict__ dst, size_t n) {
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(src[i], &dst[i]);
}

__global__ __launch_bounds__(256) void soa31_kernel(const float* __restrict__ src,
                                                    float* __restrict__ dst, int nx, int ny,
                                                    int pitch, int rows) {
    const int tiles_x = (nx + 63) / 64;
    const int x0 = (blockIdx.x % tiles_x) * 64;
    const int y0 = (blockIdx.x / tiles_x) * rows;
    const int x = x0 + (threadIdx.x & 63);
    if (x >= nx) return;
    const int w = threadIdx.x >> 6;
    const long npad = long(ny) * pitch;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    for (int y = y0 + w; y < y0 + rows && y < ny; y += 4) {
        const long rm = long(y == 0 ? ny - 1 : y - 1) * pitch, r0 = long(y) * pitch;
        const long rp = long(y == ny - 1 ? 0 : y + 1) * pitch;
        float v[31];
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int k = q % 9;
            const long r = PEY[k] > 0 ? rm : (PEY[k] < 0 ? rp : r0);   // row of y - e_ky
            const int c = PEX[k] > 0 ? xm : (PEX[k] < 0 ? xp : x);     // column of x - e_kx
            v[q] = src[q * npad + r + c];
        }
#pragma unroll
        for (int q = 27; q < 31; ++q) v[q] = src[q * npad + r0 + x];
#pragma unroll
        for (int q = 0; q < 31; ++q) __builtin_nontemporal_store(v[q] * 0.5f, &dst[q * npad + r0 + x]);
    }
}

}  // namespace
}  // namespace tlb

using namespace tlb;

extern "C" tlb_status tlb_probe_bandwidth(int kind, int nx, int ny, int tile_rows,
                                          const void* dev_src, void* dev_dst, size_t bytes,
                                          void* hip_stream, int reps, double* ms_per_launch) {
    if (!dev_src || !dev_dst || !ms_per_launch || reps <= 0) return TLB_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (kind == 0) {
        if (bytes < 16 || bytes % 16) return TLB_EINVAL;
    } else if (kind == 1) {
        if (nx < 3 || ny < 3 || tile_rows < 4 || tile_rows % 4) return TLB_EINVAL;
        const size_t pitch = (size_t(nx) + 63) / 64 * 64;
        if (bytes < 31 * pitch * size_t(ny) * 4) return TLB_EINVAL;
    } else {
        return TLB_EINVAL;
    }
    auto launch = [&]() {
        if (kind == 0) {
            hipLaunchKernelGGL(copy16_kernel, dim3(1024), dim3(256), 0, s,
                               static_cast<const f4*>(dev_src), static_cast<f4*>(dev_dst),
                               bytes / 16);
        } else {
            const int pitch = (nx + 63) / 64 * 64;
            const int tiles = ((nx + 63) / 64) * ((ny + tile_rows - 1) / tile_rows);
            hipLaunchKernelGGL(soa31_kernel, dim3(tiles), dim3(256), 0, s,
                               static_cast<const float*>(dev_src), static_cast<float*>(dev_dst), nx,
                               ny, pitch, tile_rows);
        }
    };
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        launch();   // warm-up
        e = hipEventRecord(a, s);
    }
    if (e == hipSuccess) {
        for (int i = 0; i < reps; ++i) launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return TLB_EDEVICE;
    *ms_per_launch = double(ms) / reps;
    return TLB_OK;
}
