// k_select.hip -- the relational selection sigma_theta(R) of eq. 3 as a
// selection vector: ascending qualifying row ids, produced at memory speed in
// two passes (the filtering step that the paper's late-materialisation
// strategy stages first, Section 3.2):
//   1. bitmap + per-block population counts (reads the attribute columns once);
//   2. per-block offset (sum of the preceding block counts, L2-resident) and
//      order-preserving compaction of the bitmap into row ids.
#include "internal.h"

namespace vrs {

// One block = SEL_BLOCK_ROWS rows = 32 steps of 256 rows; every wave turns
// 64 predicate results into one 64-bit ballot.
__global__ __launch_bounds__(256) void select_bitmap_kernel(const int32_t *__restrict__ attr,
                                                            int64_t n, int64_t an, PredDev p,
                                                            uint32_t *__restrict__ bitmap,
                                                            uint32_t *__restrict__ blkcnt) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * SEL_BLOCK_ROWS;
    uint32_t mycount = 0;
    for (int step = 0; step < SEL_BLOCK_ROWS / 256; ++step) {
        int64_t row0 = base + step * 256 + wave * 64;
        int64_t row = row0 + lane;
        bool q = row < n && pred_eval(p, attr, an, row);
        uint64_t m = __ballot(q);
        if (lane == 0 && row0 < n) {
            int64_t w = row0 >> 5;  // row0 is a multiple of 64
            bitmap[w] = (uint32_t)m;
            if (row0 + 32 < n) bitmap[w + 1] = (uint32_t)(m >> 32);
            mycount += (uint32_t)__popcll(m);
        }
    }
    __shared__ uint32_t wc[4];
    if (lane == 0) wc[wave] = mycount;
    __syncthreads();
    if (threadIdx.x == 0) blkcnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ __launch_bounds__(256) void select_ids_kernel(const uint32_t *__restrict__ bitmap,
                                                         const uint32_t *__restrict__ blkcnt,
                                                         int64_t n, int nblk,
                                                         int32_t *__restrict__ ids,
                                                         int64_t *__restrict__ count) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ uint64_t red[256];
    __shared__ uint32_t wtot[4];
    // offset of this block = sum of the counts of all earlier blocks
    uint64_t part = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += 256) part += blkcnt[j];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    uint64_t off = red[0];
    const int64_t base = (int64_t)blockIdx.x * SEL_BLOCK_ROWS;
    for (int step = 0; step < SEL_BLOCK_ROWS / 256; ++step) {
        int64_t row = base + step * 256 + threadIdx.x;
        bool q = false;
        if (row < n) q = (bitmap[row >> 5] >> (row & 31)) & 1u;
        uint64_t m = __ballot(q);
        uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t wo = 0;
        for (int w = 0; w < wave; ++w) wo += wtot[w];
        if (q) ids[off + wo + below] = (int32_t)row;
        off += wtot[0] + wtot[1] + wtot[2] + wtot[3];
        __syncthreads();
    }
    if (blockIdx.x == (unsigned)nblk - 1 && threadIdx.x == 0) *count = (int64_t)off;
}

hipError_t launch_select(const int32_t *attr, int64_t n, int64_t an, const PredDev &p,
                         uint32_t *bitmap, uint32_t *blkcnt, int32_t *ids, int64_t *count,
                         hipStream_t s) {
    int nblk = (int)((n + SEL_BLOCK_ROWS - 1) / SEL_BLOCK_ROWS);
    select_bitmap_kernel<<<nblk, 256, 0, s>>>(attr, n, an, p, bitmap, blkcnt);
    select_ids_kernel<<<nblk, 256, 0, s>>>(bitmap, blkcnt, n, nblk, ids, count);
    return hipGetLastError();
}

}  // namespace vrs
