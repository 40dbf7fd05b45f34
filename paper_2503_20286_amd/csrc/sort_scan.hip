// Stable LSD radix sort of (uint64 key, uint32 value) pairs and ordered
// stream compaction of a byte flag array.  Both are used by the selection
// pipeline: the sort orders the points by their exact key sum (a linear
// extension of Pareto dominance); the compaction emits the selected indices
// in ascending order (Eq. (13)).
#include "kernels.h"
#include "prims.h"

namespace nsga3 {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;  // keys per block
constexpr int kCmpTile = 256 * 8;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                        int shift, uint32_t *__restrict__ hist,
                                                        int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const int64_t p = base + it * kRsThreads + threadIdx.x;
        if (p < n) atomicAdd(&h[(uint32_t)(keys[p] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];  // block-major
}

// Exclusive scan of `n` uint32 values in place, one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_inplace(uint32_t *__restrict__ v, int64_t n,
                                                       uint32_t *__restrict__ total) {
    __shared__ uint32_t lds[17];
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t s0 = (int64_t)threadIdx.x * per;
    const int64_t s1 = s0 + per < n ? s0 + per : n;
    uint32_t sum = 0;
    for (int64_t i = s0; i < s1; ++i) sum += v[i];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(sum, lds, &tot);
    for (int64_t i = s0; i < s1; ++i) {
        uint32_t t = v[i];
        v[i] = run;
        run += t;
    }
    if (total && threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                           const uint32_t *__restrict__ vin,
                                                           uint64_t *__restrict__ kout,
                                                           uint32_t *__restrict__ vout, int64_t n,
                                                           int shift,
                                                           const uint32_t *__restrict__ offs,
                                                           int nblocks) {
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[kRsThreads / kWave][256];
    __shared__ uint32_t scan_lds[17];
    const uint32_t tid = threadIdx.x;
    const uint32_t w = tid / kWave;
    // Offsets of this block's digits: all keys with a smaller digit, plus keys
    // with the same digit in earlier blocks.  The histogram (digit-major) is
    // read cooperatively and summed with LDS atomics.
    {
        // thread = digit: sum the digit's counts over all blocks and over the
        // blocks before this one (block-major histogram: coalesced rows)
        uint32_t before = 0, total = 0;
        int b = 0;
        for (; b + 4 <= nblocks; b += 4) {
            const uint32_t h0 = offs[(size_t)(b + 0) * 256 + tid];
            const uint32_t h1 = offs[(size_t)(b + 1) * 256 + tid];
            const uint32_t h2 = offs[(size_t)(b + 2) * 256 + tid];
            const uint32_t h3 = offs[(size_t)(b + 3) * 256 + tid];
            total += h0 + h1 + h2 + h3;
            before += (b + 0 < (int)blockIdx.x ? h0 : 0u) + (b + 1 < (int)blockIdx.x ? h1 : 0u) +
                      (b + 2 < (int)blockIdx.x ? h2 : 0u) + (b + 3 < (int)blockIdx.x ? h3 : 0u);
        }
        for (; b < nblocks; ++b) {
            const uint32_t h = offs[(size_t)b * 256 + tid];
            total += h;
            before += b < (int)blockIdx.x ? h : 0u;
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(total, scan_lds, &tot);
        base_off[tid] = ex + before;
        run[tid] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int it = 0; it < kRsItems; ++it) {
#pragma unroll
        for (int q = 0; q < kRsThreads / kWave; ++q) wc[q][tid] = 0;
        __syncthreads();
        const int64_t p = base + it * kRsThreads + tid;
        const bool valid = p < n;
        const uint64_t key = valid ? kin[p] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t m = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = ballot(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t below = lanes_below(m);
        const uint32_t cnt = (uint32_t)__popcll(m);
        if (valid && below == cnt - 1) wc[w][d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t pre = run[d];
            for (uint32_t q = 0; q < w; ++q) pre += wc[q][d];
            const uint32_t dst = base_off[d] + pre + below;
            kout[dst] = key;
            vout[dst] = vin[p];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < kRsThreads / kWave; ++q) add += wc[q][tid];
        run[tid] += add;
        __syncthreads();
    }
}

size_t radix_sort_temp_bytes(int64_t n) {
    const int64_t nb = (n + kRsTile - 1) / kRsTile;
    return (size_t)(256 * nb + 64) * sizeof(uint32_t);
}

// Sorts keys[0..n) (with values) on bits [0, nbits) in 8-bit digits.  Uses
// (k_alt, v_alt) as ping-pong buffers; the result lands in (keys, vals) when
// the number of passes is even, else in the alternates: *in_alt reports which.
void radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *k_alt, uint32_t *v_alt, int64_t n,
                      int nbits, uint32_t *temp, hipStream_t s, bool *in_alt) {
    const int nb = (int)((n + kRsTile - 1) / kRsTile);
    uint64_t *ka = keys, *kb = k_alt;
    uint32_t *va = vals, *vb = v_alt;
    int passes = 0;
    for (int shift = 0; shift < nbits; shift += 8, ++passes) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kRsThreads), 0, s, ka, n, shift, temp, nb);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kRsThreads), 0, s, ka, va, kb, vb, n,
                           shift, temp, nb);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    *in_alt = (passes & 1) != 0;
}

// ---------------------------------------------------------------------------
// Ordered compaction: out[...] = ascending indices i with flag[i] != 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cmp_count(const uint8_t *__restrict__ flag, int64_t n,
                                                   uint32_t *__restrict__ blk) {
    __shared__ uint32_t lds[5];
    const int64_t base = (int64_t)blockIdx.x * kCmpTile;
    uint32_t c = 0;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int64_t p = base + it * 256 + threadIdx.x;
        if (p < n && flag[p]) ++c;
    }
    c = wave_sum(c);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

__global__ __launch_bounds__(256) void k_cmp_write(const uint8_t *__restrict__ flag, int64_t n,
                                                   const uint32_t *__restrict__ blkoff,
                                                   int32_t *__restrict__ out, int64_t cap) {
    __shared__ uint32_t lds[17];
    const int64_t base = (int64_t)blockIdx.x * kCmpTile;
    uint32_t off = blkoff[blockIdx.x];
    for (int it = 0; it < 8; ++it) {
        const int64_t p = base + it * 256 + threadIdx.x;
        const uint32_t f = (p < n && flag[p]) ? 1u : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(f, lds, &tot);
        if (f && (int64_t)(off + ex) < cap) out[off + ex] = (int32_t)p;
        off += tot;
    }
}

void scan_inplace(uint32_t *v, int64_t n, uint32_t *total, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, v, n, total);
}

size_t compact_temp_bytes(int64_t n) {
    return (size_t)((n + kCmpTile - 1) / kCmpTile + 64) * sizeof(uint32_t);
}

void compact_flags(const uint8_t *flag, int64_t n, int32_t *out, int64_t cap, uint32_t *temp,
                   uint32_t *total, hipStream_t s) {
    const int nb = (int)((n + kCmpTile - 1) / kCmpTile);
    hipLaunchKernelGGL(k_cmp_count, dim3(nb), dim3(256), 0, s, flag, n, temp);
    hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, temp, (int64_t)nb, total);
    hipLaunchKernelGGL(k_cmp_write, dim3(nb), dim3(256), 0, s, flag, n, temp, out, cap);
}

}  // namespace nsga3
