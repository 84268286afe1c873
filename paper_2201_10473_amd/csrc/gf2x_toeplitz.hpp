// gf2x_toeplitz.hpp -- shared-operand batches h * r_i mod (X^n - 1) as one
// circulant-matrix product on int8 MFMA (the circulant / ring isomorphism of
// Section 1).  Host interface used by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gf2x.h"

namespace gf2x {
namespace toeplitz {

struct Workspace {
    void *buf = nullptr;       // device scratch: bit image of h and item offsets
    size_t bytes = 0;
    hipEvent_t done = nullptr; // recorded after the last launch that read buf
    bool used = false;
};

// Shape constants shared with the host driver.
constexpr int kRowsWG = 256;    // output bits per workgroup
constexpr int kColsWG = 64;     // batch items per workgroup
constexpr int kStepBits = 128;  // K bits per step
constexpr int kColStride = 36;  // dwords per item row of the spread tile (32 + pad)
constexpr int kTileDwords = kColsWG * kColStride;

// h = a_base + items[0].a_off shared by all items; r_i = b_base + items[i].b_off;
// c_base + items[i].c_off receives h * r_i mod (X^n - 1).
int run(Workspace &ws, size_t budget, size_t &allocated, const gf2x_item *items, uint32_t count,
        uint64_t *c_base, const uint64_t *a_base, const uint64_t *b_base, int num_cu, hipStream_t s);
void release(Workspace &ws);
const char *last_error();

}  // namespace toeplitz
}  // namespace gf2x
