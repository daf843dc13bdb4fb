// k_select.hip -- the relational selection sigma_theta(R) of eq. 3 as a
// selection vector: ascending qualifying row ids, produced at memory speed in
// two passes (the filtering step that the paper's late-materialisation
// strategy stages first, Section 3.2):
//   1. bitmap + per-block population counts (reads the attribute columns once);
//   2. per-block offset (sum of the preceding block counts, L2-resident) and
//      order-preserving compaction of the bitmap into row ids.
// Both passes issue every load of a block before they use any of them, so a
// block keeps its whole share of the columns in flight.
#include "internal.h"

namespace vrs {

constexpr int SEL_STEPS = SEL_BLOCK_ROWS / 256;  // 256-row steps per block

// One block = SEL_BLOCK_ROWS rows = SEL_STEPS steps of 256 rows; row
// base + s * 256 + tid belongs to thread tid at step s.  Every wave turns a
// step's 64 predicate results into one 64-bit ballot.  NT = number of terms
// (the loads of all terms and steps are issued together).
template <int NT>
__global__ __launch_bounds__(256) void select_bitmap_kernel(const int32_t *__restrict__ attr,
                                                            int64_t n, int64_t an, PredDev p,
                                                            uint32_t *__restrict__ bitmap,
                                                            uint32_t *__restrict__ blkcnt) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * SEL_BLOCK_ROWS + threadIdx.x;
    bool q[SEL_STEPS];
    if (NT == 0) {
#pragma unroll
        for (int s = 0; s < SEL_STEPS; ++s) q[s] = p.nterms == 0 && base + s * 256 < n;
    } else {
        int32_t v[NT > 0 ? NT : 1][SEL_STEPS];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int32_t *col = attr + (int64_t)p.col[t] * an;
#pragma unroll
            for (int s = 0; s < SEL_STEPS; ++s) {
                const int64_t row = base + s * 256;
                v[t][s] = row < n ? col[row] : 0;
            }
        }
#pragma unroll
        for (int s = 0; s < SEL_STEPS; ++s) {
            bool ok = base + s * 256 < n;
#pragma unroll
            for (int t = 0; t < NT; ++t) ok = ok && v[t][s] >= p.lo[t] && v[t][s] <= p.hi[t];
            q[s] = ok;
        }
    }
    // step s's 64-bit mask goes to lane s, and the wave's 32 masks are
    // written by one store instruction (instead of 64 single-lane stores)
    static_assert(SEL_STEPS <= 64, "one lane per step");
    uint32_t mycount = 0;
    uint64_t mine = 0;
#pragma unroll
    for (int s = 0; s < SEL_STEPS; ++s) {
        const uint64_t m = __ballot(q[s]);
        mine = lane == s ? m : mine;
        mycount += (uint32_t)__popcll(m);  // (rows past n never qualify)
    }
    {
        const int64_t row0 = (int64_t)blockIdx.x * SEL_BLOCK_ROWS + lane * 256 + wave * 64;
        if (lane < SEL_STEPS && row0 < n) {
            const int64_t w = row0 >> 5;  // row0 is a multiple of 64
            if (row0 + 32 < n)
                *(uint2 *)(bitmap + w) = make_uint2((uint32_t)mine, (uint32_t)(mine >> 32));
            else
                bitmap[w] = (uint32_t)mine;
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
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ uint64_t red[256];
    __shared__ uint32_t pre[SEL_STEPS * 4];  // ids before (step, wave) within the block
    const int64_t base = (int64_t)blockIdx.x * SEL_BLOCK_ROWS + tid;
    // this thread's bits, one per step (all words requested together)
    uint32_t wd[SEL_STEPS];
#pragma unroll
    for (int s = 0; s < SEL_STEPS; ++s) {
        const int64_t row = base + s * 256;
        wd[s] = row < n ? bitmap[row >> 5] : 0u;
    }
    // offset of this block = sum of the counts of all earlier blocks
    uint64_t part = 0;
    for (int j = tid; j < (int)blockIdx.x; j += 256) part += blkcnt[j];
    red[tid] = part;
    uint64_t m[SEL_STEPS];
#pragma unroll
    for (int s = 0; s < SEL_STEPS; ++s) {
        const int64_t row = base + s * 256;
        m[s] = __ballot(row < n && ((wd[s] >> (row & 31)) & 1u));
        if (lane == 0) pre[s * 4 + wave] = (uint32_t)__popcll(m[s]);
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const uint64_t off = red[0];
    // exclusive scan of the SEL_STEPS * 4 = 128 (step, wave) counts, in row
    // order: an inclusive scan inside each of the first two waves (lane
    // shuffles), then the first wave's total added to the second's
    static_assert(SEL_STEPS * 4 == 128, "two waves scan the step counts");
    __shared__ uint32_t wtot;
    uint32_t c = 0, inc = 0;
    if (tid < 128) {
        c = pre[tid];
        inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (tid == 63) wtot = inc;
    }
    __syncthreads();
    if (tid < 128) {
        const uint32_t ex = inc - c + (tid >= 64 ? wtot : 0u);
        pre[tid] = ex;
        if (tid == 127 && blockIdx.x == (unsigned)nblk - 1) *count = (int64_t)(off + ex + c);
    }
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int s = 0; s < SEL_STEPS; ++s) {
        if ((m[s] >> lane) & 1ull)
            ids[off + pre[s * 4 + wave] + (uint32_t)__popcll(m[s] & lt)] = (int32_t)(base + s * 256);
    }
}

hipError_t launch_select(const int32_t *attr, int64_t n, int64_t an, const PredDev &p,
                         uint32_t *bitmap, uint32_t *blkcnt, int32_t *ids, int64_t *count,
                         hipStream_t s) {
    int nblk = (int)((n + SEL_BLOCK_ROWS - 1) / SEL_BLOCK_ROWS);
    switch (p.nterms < 0 ? 0 : p.nterms) {
    case 0: select_bitmap_kernel<0><<<nblk, 256, 0, s>>>(attr, n, an, p, bitmap, blkcnt); break;
    case 1: select_bitmap_kernel<1><<<nblk, 256, 0, s>>>(attr, n, an, p, bitmap, blkcnt); break;
    case 2: select_bitmap_kernel<2><<<nblk, 256, 0, s>>>(attr, n, an, p, bitmap, blkcnt); break;
    case 3: select_bitmap_kernel<3><<<nblk, 256, 0, s>>>(attr, n, an, p, bitmap, blkcnt); break;
    default: select_bitmap_kernel<4><<<nblk, 256, 0, s>>>(attr, n, an, p, bitmap, blkcnt); break;
    }
    select_ids_kernel<<<nblk, 256, 0, s>>>(bitmap, blkcnt, n, nblk, ids, count);
    return hipGetLastError();
}

}  // namespace vrs
