// gf2x_toeplitz.hip -- kernels and host driver of the shared-operand path
// (the tile itself is in gf2x_toeplitz_device.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gf2x_toeplitz.hpp"
#include "gf2x_toeplitz_device.hpp"

namespace gf2x {
namespace toeplitz {

__global__ void k_prepare_hr(const uint64_t *h, u32 n, u32 P, u32 *hr, u32 hr_dwords) {
    const u32 d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < hr_dwords) hr[d] = hr_dword(h, n, P, d);
}

__global__ __launch_bounds__(256) void k_toeplitz(const u32 *hr, u32 hr_dwords, u32 n, u32 P,
                                                  const uint64_t *r_base, const uint64_t *b_off,
                                                  uint64_t *c_base, const uint64_t *c_off, u32 count) {
    extern __shared__ u32 lds[];
    toeplitz_tile(hr, hr_dwords, n, P, r_base, b_off, c_base, c_off, count, blockIdx.x, blockIdx.y, lds);
}

// ------------------------------------------------------------------ host
namespace {
thread_local std::string g_err;

int dev_err(hipError_t e) {
    g_err = std::string(hipGetErrorName(e)) + ": " + hipGetErrorString(e);
    return GF2X_EDEVICE;
}
}  // namespace

const char *last_error() { return g_err.c_str(); }

void release(Workspace &ws) {
    if (ws.buf) hipFree(ws.buf);
    if (ws.done) hipEventDestroy(ws.done);
    ws.buf = nullptr;
    ws.done = nullptr;
    ws.bytes = 0;
    ws.used = false;
}

int run(Workspace &ws, size_t budget, size_t &allocated, const gf2x_item *items, uint32_t count,
        uint64_t *c_base, const uint64_t *a_base, const uint64_t *b_base, int num_cu, hipStream_t s) {
    (void)num_cu;
    const u32 n = items[0].n_bits;
    const u32 W = (n + 63u) / 64u;
    const u32 steps = (n + kStepBits - 1) / kStepBits;
    const u32 rows = (n + kRowsWG - 1) / kRowsWG * kRowsWG;
    const u32 P = rows + 64u;
    const u32 hr_bits = P + steps * kStepBits + 128u;
    const u32 hr_dwords = (hr_bits + 31u) / 32u + 2u;
    const size_t need = (size_t)hr_dwords * 4 + (size_t)count * 16 + 256;
    hipError_t e;
    if (!ws.done) {
        e = hipEventCreateWithFlags(&ws.done, hipEventDisableTiming);
        if (e != hipSuccess) return dev_err(e);
    }
    if (ws.used) {
        e = hipStreamWaitEvent(s, ws.done, 0);
        if (e != hipSuccess) return dev_err(e);
    }
    if (need > ws.bytes) {
        if (allocated - ws.bytes + need > budget) return GF2X_ENOMEM;
        if (ws.buf) {
            e = hipEventSynchronize(ws.done);
            if (e != hipSuccess) return dev_err(e);
            hipFree(ws.buf);
            allocated -= ws.bytes;
            ws.buf = nullptr;
            ws.bytes = 0;
        }
        if (hipMalloc(&ws.buf, need) != hipSuccess) return GF2X_ENOMEM;
        ws.bytes = need;
        allocated += need;
    }
    u32 *hr = reinterpret_cast<u32 *>(ws.buf);
    uint64_t *offs = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(ws.buf) + ((size_t)hr_dwords * 4 + 255) / 256 * 256);
    std::vector<uint64_t> host(2 * (size_t)count);
    for (uint32_t i = 0; i < count; ++i) {
        host[i] = items[i].b_off;
        host[count + i] = items[i].c_off;
    }
    e = hipMemcpyAsync(offs, host.data(), host.size() * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return dev_err(e);
    hipLaunchKernelGGL(k_prepare_hr, dim3((hr_dwords + 255) / 256), dim3(256), 0, s, a_base + items[0].a_off, n, P, hr,
                       hr_dwords);
    e = hipGetLastError();
    if (e != hipSuccess) return dev_err(e);
    // LDS: the hr window (at most steps*4 + 16 dwords) and two spread tiles
    const u32 hr_len_max = (kRowsWG + kStepBits * steps + 96u + 64u) / 32u + 4u;
    const int lds = (int)(((hr_len_max + 3u) & ~3u) + 2u * kTileDwords) * 4;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_toeplitz), hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds);
    if (e != hipSuccess) return dev_err(e);
    dim3 grid(rows / kRowsWG, (count + kColsWG - 1) / kColsWG);
    hipLaunchKernelGGL(k_toeplitz, grid, dim3(256), lds, s, hr, hr_dwords, n, P, b_base, offs, c_base, offs + count,
                       count);
    e = hipGetLastError();
    if (e != hipSuccess) return dev_err(e);
    e = hipEventRecord(ws.done, s);
    if (e != hipSuccess) return dev_err(e);
    ws.used = true;
    (void)W;
    return GF2X_OK;
}

}  // namespace toeplitz
}  // namespace gf2x
