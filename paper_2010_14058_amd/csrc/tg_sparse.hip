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

// Neighbours above the row's own id (rows sorted): its canonical edges.
__global__ void k_upper_count(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                              int64_t n, int64_t *__restrict__ cnt) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u == 0) cnt[n] = 0;
    if (u >= n) return;
    cnt[u] = rp[u + 1] - upper_bound(col, rp[u], rp[u + 1], (int32_t)u);
}

// One wave per row: the row's canonical edges (u, x), x > u, at eoff[u] on.
__global__ void k_edge_list(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                            int64_t n, const int64_t *__restrict__ eoff,
                            int64_t *__restrict__ uv, const uint32_t *__restrict__ status) {
    if (input_failed(status)) return;
    const int lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; u < n;
         u += nwaves) {
        const int64_t first = rp[u + 1] - (eoff[u + 1] - eoff[u]);
        for (int64_t s = first + lane; s < rp[u + 1]; s += WAVE) {
            const int64_t e = eoff[u] + (s - first);
            uv[2 * e] = u;
            uv[2 * e + 1] = col[s];
        }
    }
}

__global__ void k_edge_count_check(const int64_t *__restrict__ eoff, int64_t n, int64_t m,
                                   uint32_t *__restrict__ status) {
    *status = eoff[n] == m ? 0u : ST_EDGE_COUNT;
}

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" {

size_t tg_edge_list_workspace_bytes(int64_t n) {
    if (n < 0) return 0;
    return 2 * (((size_t)(n + 2) * sizeof(int64_t) + 255) / 256 * 256) + scan_tmp_bytes(n + 1) +
           256;
}

tg_status tg_edge_list(const int64_t *row_ptr, const int32_t *col, int64_t n, int64_t nnz,
                       int64_t *edge_uv, void *workspace, size_t ws_bytes, void *stream) {
    if (n < 0 || nnz < 0 || (nnz & 1) || (n > 0 && !row_ptr) || (nnz > 0 && (!col || !edge_uv)) ||
        !workspace || ((uintptr_t)workspace & 255u))
        return TG_E_INVALID_ARG;
    if (ws_bytes < tg_edge_list_workspace_bytes(n)) return TG_E_WORKSPACE;
    if (n == 0 || nnz == 0) return TG_OK;
    hipStream_t st = (hipStream_t)stream;
    const size_t arr = ((size_t)(n + 2) * sizeof(int64_t) + 255) / 256 * 256;
    char *w = static_cast<char *>(workspace);
    int64_t *cnt = reinterpret_cast<int64_t *>(w);
    int64_t *eoff = reinterpret_cast<int64_t *>(w + arr);
    uint32_t *status = reinterpret_cast<uint32_t *>(w + 2 * arr);
    int64_t *tmp = reinterpret_cast<int64_t *>(w + 2 * arr + 256);
    k_upper_count<<<(unsigned)((n + 256) / 256), 256, 0, st>>>(row_ptr, col, n, cnt);
    if (hipGetLastError() != hipSuccess) return TG_E_DEVICE;
    if (launch_excl_scan(cnt, eoff, n + 1, tmp, nullptr, st) != hipSuccess) return TG_E_DEVICE;
    k_edge_count_check<<<1, 1, 0, st>>>(eoff, n, nnz / 2, status);
    k_edge_list<<<row_blocks(n), 256, 0, st>>>(row_ptr, col, n, eoff, edge_uv, status);
    if (hipGetLastError() != hipSuccess) return TG_E_DEVICE;
    uint32_t bits = 0;
    if (hipMemcpyAsync(&bits, status, sizeof(bits), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return TG_E_DEVICE;
    return bits ? TG_E_NOT_SIMPLE : TG_OK;
}

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
