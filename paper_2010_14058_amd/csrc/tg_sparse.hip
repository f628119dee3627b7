// Sparse per-edge output (Sec. 4.6): each edge keeps only its nonzero
// (column, count) pairs, columns ascending, edges in canonical order, with a
// per-edge offset array.  Built from the dense per-edge table in two passes
// (nonzeros per edge + prefix sum, then the fill), so the layout is a pure
// function of the dense table.
#include <hip/hip_runtime.h>

#include "tg_device.hpp"

namespace tg {
namespace {

// One wave per edge row (grid-stride): number of nonzero entries.
__global__ void __launch_bounds__(256) k_row_nnz(const uint64_t *__restrict__ rows, int64_t m, int W,
                                                 int64_t *__restrict__ cnt) {
    const int lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[m] = 0;  // the scan's last element: the total
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; e < m;
         e += nwaves) {
        const uint64_t *row = rows + (size_t)e * W;
        int64_t c = 0;
        for (int q0 = 0; q0 < W; q0 += WAVE) {
            const int q = q0 + lane;
            const bool nz = q < W && row[q] != 0ull;
            c += __popcll(__ballot(nz));
        }
        if (lane == 0) cnt[e] = c;
    }
}

// One wave per edge row (grid-stride): its nonzero entries at the edge's
// offset.
__global__ void __launch_bounds__(256) k_row_fill(const uint64_t *__restrict__ rows, int64_t m, int W,
                                                  const int64_t *__restrict__ off,
                                                  uint16_t *__restrict__ keys,
                                                  uint64_t *__restrict__ counts) {
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; e < m;
         e += nwaves) {
        const uint64_t *row = rows + (size_t)e * W;
        int64_t pos = off[e];
        for (int q0 = 0; q0 < W; q0 += WAVE) {
            const int q = q0 + lane;
            const uint64_t v = q < W ? row[q] : 0ull;
            const uint64_t bal = __ballot(v != 0ull);
            if (v) {
                const int64_t at = pos + __popcll(bal & below);
                keys[at] = (uint16_t)q;
                counts[at] = v;
            }
            pos += __popcll(bal);
        }
    }
}

// Workgroups for a grid-stride launch over `waves` rows, four waves a
// workgroup: enough to fill the device, no more.
unsigned row_blocks(int64_t waves) {
    int64_t b = (waves + 3) / 4;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0 && b > (int64_t)cus * 32)
        b = (int64_t)cus * 32;
    return b > 0 ? (unsigned)b : 1u;
}

// Tile sums of the prefix sum over m + 1 entries.
size_t scan_tmp_bytes(int64_t m) { return (size_t)(scan_tiles(m + 1) + 1) * sizeof(int64_t); }

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" {

size_t tg_sparse_workspace_bytes(int64_t m) {
    if (m < 0) return 0;
    return ((size_t)(m + 1) * sizeof(int64_t) + 255) / 256 * 256 + scan_tmp_bytes(m);
}

tg_status tg_sparse_offsets(const uint64_t *rows, int64_t m, int32_t L, int64_t *edge_off,
                            void *workspace, size_t ws_bytes, void *stream) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (m < 0 || !edge_off || (m > 0 && !rows) || !workspace)
        return TG_E_INVALID_ARG;
    const size_t need = tg_sparse_workspace_bytes(m);
    if (ws_bytes < need) return TG_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const int W = tg_row_width(L);
    int64_t *cnt = static_cast<int64_t *>(workspace);
    const size_t cnt_bytes = ((size_t)(m + 1) * sizeof(int64_t) + 255) / 256 * 256;
    int64_t *tmp = reinterpret_cast<int64_t *>(static_cast<char *>(workspace) + cnt_bytes);
    k_row_nnz<<<row_blocks(m), 256, 0, st>>>(rows, m, W, cnt);
    if (hipGetLastError() != hipSuccess) return TG_E_DEVICE;
    if (launch_excl_scan(cnt, edge_off, m + 1, tmp, nullptr, st) != hipSuccess) return TG_E_DEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? TG_OK : TG_E_DEVICE;
}

tg_status tg_sparse_fill(const uint64_t *rows, int64_t m, int32_t L, const int64_t *edge_off,
                         uint16_t *keys, uint64_t *counts, void *stream) {
    if (L < 1 || L > TG_MAX_L) return TG_E_L_RANGE;
    if (m < 0 || !edge_off || (m > 0 && (!rows || !keys || !counts)))
        return TG_E_INVALID_ARG;
    if (m == 0) return TG_OK;
    hipStream_t st = (hipStream_t)stream;
    const int W = tg_row_width(L);
    k_row_fill<<<row_blocks(m), 256, 0, st>>>(rows, m, W, edge_off, keys, counts);
    if (hipGetLastError() != hipSuccess) return TG_E_DEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? TG_OK : TG_E_DEVICE;
}

}  // extern "C"
