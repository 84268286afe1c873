// gf2x_toeplitz.hip -- placeholder until the MFMA kernel lands.
#include "gf2x_toeplitz.hpp"

namespace gf2x {
namespace toeplitz {

int run(Workspace &, size_t, size_t &, const gf2x_item *, uint32_t, uint64_t *, const uint64_t *,
        const uint64_t *, int, hipStream_t) {
    return GF2X_ENOTSUP;
}
void release(Workspace &ws) {
    if (ws.buf) hipFree(ws.buf);
    ws.buf = nullptr;
    ws.bytes = 0;
}
const char *last_error() { return ""; }

}  // namespace toeplitz
}  // namespace gf2x
