// Device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// Radix sort: stable LSD with up to 8-bit digits over a fixed grid of
// blocks (described below).
#include "bgs_internal.h"

namespace bgs {

namespace {

__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += t;
    }
    return v;
}

// Exclusive scan over the 256 threads of a block; lds needs 4 words.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t x = lds[w];
        if ((uint32_t)w < wave) off += x;
        tot += x;
    }
    __syncthreads();
    if (total) *total = tot;
    return off + inc - v;
}

__device__ inline uint32_t block_sum(uint32_t v, uint32_t* lds) {
    uint32_t tot;
    block_excl_scan(v, lds, &tot);
    return tot;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                     const uint32_t* __restrict__ idx,
                                                     const uint32_t* __restrict__ n_dev, int64_t n_cap,
                                                     uint32_t* __restrict__ partials) {
    __shared__ uint32_t lds[4];
    const int64_t n = n_dev ? (int64_t)*n_dev : n_cap;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j * 256 + threadIdx.x;
        if (i < n) s += in[idx ? idx[i] : i];
    }
    uint32_t tot = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// `in` and `out` may be the same array (in-place scan): every thread reads
// its own elements before the block-wide scan and writes them after it.
__global__ __launch_bounds__(256) void k_scan_down(const uint32_t* in, const uint32_t* __restrict__ idx,
                                                   const uint32_t* __restrict__ n_dev, int64_t n_cap,
                                                   const uint32_t* partials, uint32_t* out) {
    __shared__ uint32_t lds[4];
    const int64_t n = n_dev ? (int64_t)*n_dev : n_cap;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        v[j] = (i < n) ? in[idx ? idx[i] : i] : 0u;
        s += v[j];
    }
    uint32_t run = block_excl_scan(s, lds, nullptr) + partials[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i <= n) out[i] = run;
        run += v[j];
    }
}

// Two-launch form for up to kScanFlat blocks: every block adds up the block
// sums before its own (at most kScanFlat / 256 loads per thread), so no
// second level is needed.  With status given, the thread that writes out[n]
// also records the total as the pass's key count, and the blocks clear the
// tile ranges (see KeyCount).
constexpr int64_t kScanFlat = 4096;

// parts: partials per block of the scan (1: one sum per block of kScanBlock
// elements; kScanItems: one per 256 elements).
__global__ __launch_bounds__(256) void k_scan_down_flat(const uint32_t* in, const uint32_t* __restrict__ idx,
                                                        const uint32_t* __restrict__ n_dev, int64_t n_cap,
                                                        const uint32_t* __restrict__ partials, int parts,
                                                        uint32_t* out, KeyCount kcnt) {
    __shared__ uint32_t lds[4];
    const int64_t n = n_dev ? (int64_t)*n_dev : n_cap;
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < kcnt.n_tiles; t += gridDim.x * 256)
        kcnt.ranges[t] = make_uint2(0u, 0u);
    uint32_t pre = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x * (uint32_t)parts; b += 256) pre += partials[b];
    pre = block_sum(pre, lds);
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        v[j] = (i < n) ? in[idx ? idx[i] : i] : 0u;
        s += v[j];
    }
    uint32_t run = block_excl_scan(s, lds, nullptr) + pre;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        int64_t i = base + j;
        if (i <= n) out[i] = run;
        if (i == n && kcnt.st) {
            DevStatus* st = kcnt.st;
            st->n_slots = 0;
            st->n_items = 0;
            st->n_keys = run;
            st->n_sort = run < kcnt.cap ? run : kcnt.cap;
            if (run > kcnt.cap) st->overflow |= 1u;
            if (kcnt.which == 0) st->n_keys_dom = run;
            else st->n_keys_roi = run;
        }
        run += v[j];
    }
}

}  // namespace

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool scan_counts(const uint32_t* in, const uint32_t* idx, uint32_t* out, int64_t n, uint32_t* tmp,
                 const KeyCount& kcnt, hipStream_t s, hipError_t* err) {
    const int64_t nb = ceil_div(n + 1, kScanBlock);
    if (nb > kScanFlat) return false;
    if (nb > 1)
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, s, in, idx, nullptr, n, tmp);
    hipLaunchKernelGGL(k_scan_down_flat, dim3((unsigned)nb), dim3(256), 0, s, in, idx, nullptr, n, tmp, 1, out,
                       kcnt);
    *err = hipGetLastError();
    return true;
}

bool scan_is_flat(int64_t n) { return ceil_div(n + 1, kScanBlock) <= kScanFlat; }

bool scan_counts_presummed(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* partials,
                           const KeyCount& kcnt, hipStream_t s, hipError_t* err) {
    const int64_t nb = ceil_div(n + 1, kScanBlock);
    if (nb > kScanFlat) return false;
    hipLaunchKernelGGL(k_scan_down_flat, dim3((unsigned)nb), dim3(256), 0, s, in, nullptr, nullptr, n, partials,
                       kScanItems, out, kcnt);
    *err = hipGetLastError();
    return true;
}

size_t scan_tmp_elems(int64_t n) {
    // Level l scans n_l elements (n_0 = n) with ceil((n_l + 1) / block)
    // blocks; its block sums are the n_{l+1} elements of the next level.
    size_t tot = 0;
    int64_t m = n;
    while (true) {
        int64_t nb = ceil_div(m + 1, kScanBlock);
        tot += (size_t)nb + 64;
        if (nb <= 1) break;
        m = nb;
    }
    return tot;
}

__global__ void k_status_reset(DevStatus* st, int full) {
    constexpr int kWords = (int)(sizeof(DevStatus) / 4);
    constexpr int kSticky = (int)(offsetof(DevStatus, sticky) / 4);
    __shared__ uint32_t keep;
    if (threadIdx.x == 0) keep = full ? 0u : (st->sticky | st->overflow);
    __syncthreads();
    uint32_t* w = reinterpret_cast<uint32_t*>(st);
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) w[i] = i == kSticky ? keep : 0u;
}

hipError_t launch_status_reset(DevStatus* st, int full, hipStream_t s) {
    static_assert(sizeof(DevStatus) % 4 == 0, "status block is made of 32-bit words");
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(128), 0, s, st, full);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* dst, int64_t n, uint32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

hipError_t launch_fill_u32(uint32_t* dst, int64_t n, uint32_t value, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 2048);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, dst, n, value);
    return hipGetLastError();
}

hipError_t exclusive_scan(const uint32_t* in, const uint32_t* idx, uint32_t* out, const uint32_t* n_dev,
                          int64_t n_cap, uint32_t* tmp, hipStream_t s) {
    const int64_t nb = ceil_div(n_cap + 1, kScanBlock);
    uint32_t* partials = tmp;
    if (nb > 1) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, s, in, idx, n_dev, n_cap, partials);
        // Scan the nb block sums in place (their own element count is nb, and
        // the extra total slot they produce is never read).
        hipError_t e = exclusive_scan(partials, nullptr, partials, nullptr, nb, tmp + nb + 64, s);
        if (e != hipSuccess) return e;
    } else {
        hipError_t e = launch_fill_u32(partials, 1, 0u, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(256), 0, s, in, idx, n_dev, n_cap, partials, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Radix sort.  Stable LSD with digits of up to 8 bits (a 32-bit key takes four
// passes, an 11-bit tile id two of 6 and 5 bits).  The grid is fixed by the
// capacity (at most kRsGrid blocks; always kRsSmallGrid for small sorts,
// which use 1024-key sub-chunks instead of 6144); block b owns the contiguous
// chunk [b C, b C + C) of the *n_dev keys, C = n / grid rounded up to 256.
// A pass is three launches (their bodies are device functions taking the
// grid and the LDS, so one launch can run either form):
//   1. k_rs_hist: per-block digit counts (LDS atomics), stored
//      digit-major: counts[d * grid + b].
//   2. k_rs_scan: one block per digit scans its row over the blocks and
//      writes the digit total.
//   3. k_rs_scatter: every block scans the digit totals, then walks its chunk
//      in sub-chunks of 6144 keys: each wave ranks its 1536 keys in 24 steps
//      of 64 (1024-key sub-chunks, 4 steps, for small sorts) with match-any
//      ballots and a per-wave LDS count per digit, the sub-chunk is
//      reordered by digit in LDS, and each digit's run (24 keys on average
//      at 8 bits) is written out contiguously.  Large sorts rank digits of
//      at most 7 bits with per-thread counters instead (k_rs_scatter_cnt).
// Blocks never wait on each other.
// ---------------------------------------------------------------------------
namespace {

constexpr int kRsMaxBits = 8;
constexpr int kRsBins = 1 << kRsMaxBits;
constexpr int kRsGrid = 1024;
// Small sorts use half the grid: a 300k-key depth sort then gives each
// block about 600 keys, and its count table and per-digit scans shrink by
// half (61.8 against 69.2 us on sphere800; 256 blocks slowed the ROI sort).
constexpr int kRsSmallGrid = 512;
// Keys per thread per sub-chunk: 24 (6144-key sub-chunks, long digit runs;
// a 6M-key tile sort then gives each block one sub-chunk, not a full and a
// partial one in turn) for large sorts; 4 (1024-key sub-chunks) for small
// ones, where a block holds only a few hundred keys and its latency is the
// sort's.
constexpr int kRsItemsBig = 24, kRsItemsSmall = 4;
// A sort whose key count is known only on the device (an ROI pass's) runs
// each pass as one histogram and one scatter launch whose blocks take the
// small form up to kRsSplitKeys keys (2.8M keys: 74 us against 87 us for
// the large form) and the large form above (k_rs_hist_dual,
// k_rs_scatter_dual).  Digits of more than 7 bits, or unaligned buffers,
// launch both forms' kernels instead, each returning at once unless the
// count is in its range.
constexpr uint32_t kRsSplitKeys = 4u << 20;
struct RsGate {
    uint32_t lo, hi;  // the kernel runs iff lo <= n <= hi
};
constexpr RsGate kRsAlways{0u, 0xFFFFFFFFu};

__device__ inline uint64_t match_digit(uint32_t d, uint64_t valid, int bits) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < kRsMaxBits; ++b) {
        if (b < bits) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
    }
    return peers;
}

// Block b's chunk: n / grid keys rounded up to a multiple of 256 (and to at
// least one key per thread).  sub (the sub-chunk size) is unused here but
// keeps the chunking tied to the kernel's instance.
__device__ inline void chunk_of(uint32_t n, uint32_t grid, uint32_t b, uint32_t sub, uint32_t* lo, uint32_t* hi) {
    (void)sub;
    const uint32_t per = (uint32_t)(((uint64_t)n + grid - 1) / grid);
    const uint64_t c = ((uint64_t)per + 255u) & ~255ull;
    const uint64_t l = min<uint64_t>((uint64_t)b * c, n);
    *lo = (uint32_t)l;
    *hi = (uint32_t)min<uint64_t>(l + c, n);
}

// The kernels' bodies take the grid they partition the keys over (G; the
// block id is blockIdx.x < G) and their LDS as one array, so that one
// kernel can run either form on a count known only on the device.
template <int kRsItems>
__device__ __forceinline__ void rs_hist_body(const uint32_t* __restrict__ keys, uint32_t n, int shift, int bits,
                                             uint32_t* __restrict__ counts, uint32_t G, uint32_t* smem) {
    constexpr int kRsSub = 256 * kRsItems;
    uint32_t* h = smem;  // kRsBins words
    const uint32_t bins = 1u << bits, mask = bins - 1u;
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t lo, hi;
    chunk_of(n, G, blockIdx.x, kRsSub, &lo, &hi);
    for (uint64_t sub = lo; sub < hi; sub += kRsSub) {
        uint32_t k[kRsItems];
#pragma unroll
        for (int it = 0; it < kRsItems; ++it) {
            const uint64_t i = sub + it * 256 + threadIdx.x;
            k[it] = i < hi ? keys[i] : 0u;
        }
        // Counts only (no ranks): one LDS add per key; lanes of a wave on
        // one digit are serialised by the LDS, which costs less than
        // matching the digits with ballots.
#pragma unroll
        for (int it = 0; it < kRsItems; ++it) {
            if (sub + it * 256 + threadIdx.x < hi) atomicAdd(&h[(k[it] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < bins) counts[(uint64_t)threadIdx.x * G + blockIdx.x] = h[threadIdx.x];
}

template <int kRsItems>
__global__ __launch_bounds__(256) void k_rs_hist(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ n_dev,
                                                 uint32_t n_host, int shift, int bits,
                                                 uint32_t* __restrict__ counts, RsGate gate) {
    __shared__ uint32_t smem[kRsBins];
    const uint32_t n = n_dev ? *n_dev : n_host;
    if (n < gate.lo || n > gate.hi) return;
    rs_hist_body<kRsItems>(keys, n, shift, bits, counts, gridDim.x, smem);
}

// One block per digit: exclusive scan of counts[d * grid .. + grid) in place;
// totals[d] = the row's sum.
// grid_big (with n_dev): the grid of the large form, used when the device
// key count exceeds kRsSplitKeys.
__global__ __launch_bounds__(256) void k_rs_scan(uint32_t* __restrict__ counts, uint32_t grid,
                                                 uint32_t* __restrict__ totals, uint32_t grid_big,
                                                 const uint32_t* __restrict__ n_dev) {
    __shared__ uint32_t lds[4];
    if (n_dev && *n_dev > kRsSplitKeys) grid = grid_big;
    uint32_t* row = counts + (uint64_t)blockIdx.x * grid;
    const uint32_t per = (grid + 255) / 256, b0 = threadIdx.x * per;
    uint32_t v[kRsGrid / 256];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kRsGrid / 256; ++j) {
        v[j] = ((uint32_t)j < per && b0 + j < grid) ? row[b0 + j] : 0u;
        sum += v[j];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(sum, lds, &tot);
#pragma unroll
    for (int j = 0; j < kRsGrid / 256; ++j) {
        if ((uint32_t)j < per && b0 + j < grid) row[b0 + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

template <int kRsItems>
__host__ __device__ constexpr int rs_scatter_lds() { return 2 * 256 * kRsItems + 7 * kRsBins + 4; }

template <int kRsItems>
__device__ __forceinline__ void rs_scatter_body(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t n,
                                                int shift, int bits, const uint32_t* __restrict__ counts,
                                                const uint32_t* __restrict__ totals, uint32_t G, uint32_t* smem) {
    constexpr int kRsSub = 256 * kRsItems;
    uint32_t* s_keys = smem;
    uint32_t* s_vals = s_keys + kRsSub;
    uint32_t* cnt0 = s_vals + kRsSub;  // [4][kRsBins]
    uint32_t* dstart = cnt0 + 4 * kRsBins;
    uint32_t* gbase = dstart + kRsBins;
    uint32_t* run = gbase + kRsBins;
    uint32_t* lds = run + kRsBins;
    const auto cnt = [&](uint32_t w) { return cnt0 + w * kRsBins; };
    const uint32_t bins = 1u << bits, mask = bins - 1u;
    const bool has_v = vout != nullptr;  // keys only (a key that carries its value) when null
    uint32_t lo, hi;
    chunk_of(n, G, blockIdx.x, kRsSub, &lo, &hi);
    if (lo >= hi) return;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint32_t dt = threadIdx.x;  // the digit this thread looks after
    {
        // run[d] = (keys of smaller digits) + (keys of digit d in earlier blocks).
        const uint32_t t = dt < bins ? totals[dt] : 0u;
        const uint32_t acc = block_excl_scan(t, lds, nullptr);
        if (dt < bins) run[dt] = acc + counts[(uint64_t)dt * G + blockIdx.x];
#pragma unroll
        for (int w = 0; w < 4; ++w) cnt(w)[dt] = 0;
    }
    __syncthreads();
    for (uint64_t sub = lo; sub < hi; sub += kRsSub) {
        uint32_t k[kRsItems], v[kRsItems], r[kRsItems];
#pragma unroll
        for (int it = 0; it < kRsItems; ++it) {
            const uint64_t i = sub + wave * (64 * kRsItems) + it * 64 + lane;
            const bool ok = i < hi;
            k[it] = ok ? kin[i] : 0u;
            v[it] = (ok && has_v) ? (vin ? vin[i] : (uint32_t)i) : 0u;
        }
#pragma unroll
        for (int it = 0; it < kRsItems; ++it) {
            const uint64_t i = sub + wave * (64 * kRsItems) + it * 64 + lane;
            const bool ok = i < hi;
            const uint32_t d = (k[it] >> shift) & mask;
            const uint64_t peers = match_digit(d, __ballot(ok), bits);
            const uint32_t c = ok ? cnt(wave)[d] : 0u;
            r[it] = ok ? c + (uint32_t)__popcll(peers & lt) : 0xFFFFFFFFu;
            __builtin_amdgcn_wave_barrier();
            if (ok && (peers & lt) == 0) cnt(wave)[d] = c + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        {
            const uint32_t c0 = cnt(0)[dt], c1 = cnt(1)[dt], c2 = cnt(2)[dt], c3 = cnt(3)[dt];
            const uint32_t tot = c0 + c1 + c2 + c3;
            const uint32_t st = block_excl_scan(tot, lds, nullptr);
            cnt(0)[dt] = st;
            cnt(1)[dt] = st + c0;
            cnt(2)[dt] = st + c0 + c1;
            cnt(3)[dt] = st + c0 + c1 + c2;
            dstart[dt] = st;
            if (dt < bins) {
                gbase[dt] = run[dt];
                run[dt] += tot;
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kRsItems; ++it) {
            if (r[it] != 0xFFFFFFFFu) {
                const uint32_t lp = cnt(wave)[(k[it] >> shift) & mask] + r[it];
                s_keys[lp] = k[it];
                if (has_v) s_vals[lp] = v[it];
            }
        }
        __syncthreads();
        const uint32_t m = (uint32_t)min<uint64_t>((uint64_t)kRsSub, hi - sub);
        for (uint32_t p = threadIdx.x; p < m; p += 256) {
            const uint32_t kk = s_keys[p];
            const uint32_t d = (kk >> shift) & mask;
            const uint32_t o = gbase[d] + (p - dstart[d]);
            if (o < n) {  // always true for consistent counts; keeps every write in bounds
                kout[o] = kk;
                if (has_v) vout[o] = s_vals[p];
            }
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < 4; ++w) cnt(w)[dt] = 0;
        __syncthreads();
    }
}

template <int kRsItems>
__global__ __launch_bounds__(256) void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                    const uint32_t* __restrict__ n_dev, uint32_t n_host, int shift,
                                                    int bits, const uint32_t* __restrict__ counts,
                                                    const uint32_t* __restrict__ totals, RsGate gate) {
    __shared__ uint32_t smem[rs_scatter_lds<kRsItems>()];
    const uint32_t n = n_dev ? *n_dev : n_host;
    if (n < gate.lo || n > gate.hi) return;
    rs_scatter_body<kRsItems>(kin, vin, kout, vout, n, shift, bits, counts, totals, gridDim.x, smem);
}

// k_rs_scatter for digits of at most 7 bits and 6144-key sub-chunks, with
// the ranks taken from per-thread digit counters instead of ballots: thread
// t holds the sub-chunk's keys [24 t, 24 t + 24) (blocked, so input order is
// (thread, item) order), counts its digits in a 16-bit LDS counter per
// (digit, thread), a raking scan of the counters in (digit, thread) order
// gives every (digit, thread) its first rank, and the thread's own count
// before each key adds the rest.  Stable, like the ballot ranking, at a
// fraction of its vector work.  The counter words are padded by one word in
// 32 so the raking threads hit distinct banks; the same LDS holds the
// reordered keys and values once the ranks are known.  (At 24 keys per
// thread a counter reaches 24 and a rank 6143: 16 bits hold both.)
// Digits of 7 bits need 64 KiB of counters, which gfx950's 160 KiB of LDS
// per workgroup holds for two workgroups per CU: a 13-bit tile id then
// takes two counter-ranked passes (7 + 6 bits) instead of a ballot-ranked
// 7-bit pass and a counter-ranked one.  Digits of at most 6 bits keep the
// 32 KiB form (four workgroups per CU without values).
constexpr int kRsCntMaxBits = 7;
__host__ __device__ constexpr int rs_cnt_words(int bits) { return (1 << bits) * 256 / 2; }  // two 16-bit counters a word
__host__ __device__ constexpr int rs_cnt_lds(int bits) { return rs_cnt_words(bits) + rs_cnt_words(bits) / 32; }  // padded
static_assert(kRsItemsBig % 4 == 0, "a thread's keys are loaded as 16-byte vectors");

__device__ __forceinline__ uint32_t cnt_slot(uint32_t w) { return w + (w >> 5); }

// The counters, then the sub-chunk's keys (and values): keys alone need no
// more LDS than the 6-bit counters, so four blocks share a CU instead of
// three.
template <bool kHasV, int kBits>
__host__ __device__ constexpr int rs_cnt_buf() {
    return rs_cnt_lds(kBits) > (kHasV ? 2 : 1) * 256 * kRsItemsBig ? rs_cnt_lds(kBits)
                                                                   : (kHasV ? 2 : 1) * 256 * kRsItemsBig;
}
template <bool kHasV, int kBits>
__host__ __device__ constexpr int rs_scatter_cnt_lds() { return rs_cnt_buf<kHasV, kBits>() + 3 * (1 << kBits) + 1 + 4; }

template <bool kHasV, int kBits>
__device__ __forceinline__ void rs_scatter_cnt_body(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                    uint32_t n, int shift, int bits,
                                                    const uint32_t* __restrict__ counts,
                                                    const uint32_t* __restrict__ totals, uint32_t G, uint32_t* smem) {
    constexpr int kItems = kRsItemsBig;
    constexpr int kSub = 256 * kItems;
    constexpr int kBins = 1 << kBits;
    constexpr int kBuf = rs_cnt_buf<kHasV, kBits>();
    uint32_t* s_buf = smem;
    uint32_t* dstart = s_buf + kBuf;  // kBins + 1
    uint32_t* gbase = dstart + kBins + 1;
    uint32_t* run = gbase + kBins;
    uint32_t* lds = run + kBins;
    uint32_t* s_keys = s_buf;
    uint32_t* s_vals = s_buf + (kHasV ? kSub : 0);  // not touched without values
    const uint32_t bins = 1u << bits, mask = bins - 1u;
    constexpr bool has_v = kHasV;  // false: keys only (a key that carries its value)
    uint32_t lo, hi;
    chunk_of(n, G, blockIdx.x, kSub, &lo, &hi);
    if (lo >= hi) return;
    const uint32_t t = threadIdx.x;
    {
        // run[d] = (keys of smaller digits) + (keys of digit d in earlier blocks).
        const uint32_t tv = t < bins ? totals[t] : 0u;
        const uint32_t acc = block_excl_scan(tv, lds, nullptr);
        if (t < bins) run[t] = acc + counts[(uint64_t)t * G + blockIdx.x];
    }
    const uint32_t rake = bins / 2;         // counter words per thread (bins * 256 / 2 words over 256 threads)
    const uint32_t nclear = cnt_slot(bins * 128u);
    for (uint64_t sub = lo; sub < hi; sub += kSub) {
        const uint32_t m = (uint32_t)min<uint64_t>((uint64_t)kSub, hi - sub);
        const uint32_t i0 = t * kItems;
        uint32_t k[kItems], v[kItems];
        if (i0 + kItems <= m) {
            const uint4* kp = reinterpret_cast<const uint4*>(kin + sub + i0);
#pragma unroll
            for (int q = 0; q < kItems / 4; ++q) {
                const uint4 x = kp[q];
                k[4 * q] = x.x; k[4 * q + 1] = x.y; k[4 * q + 2] = x.z; k[4 * q + 3] = x.w;
            }
            if (has_v && vin) {
                const uint4* vp = reinterpret_cast<const uint4*>(vin + sub + i0);
#pragma unroll
                for (int q = 0; q < kItems / 4; ++q) {
                    const uint4 x = vp[q];
                    v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
                }
            } else {
#pragma unroll
                for (int it = 0; it < kItems; ++it) v[it] = (uint32_t)(sub + i0 + it);
            }
        } else {
#pragma unroll
            for (int it = 0; it < kItems; ++it) {
                const bool ok = i0 + it < m;
                k[it] = ok ? kin[sub + i0 + it] : 0u;
                v[it] = ok ? (has_v && vin ? vin[sub + i0 + it] : (uint32_t)(sub + i0 + it)) : 0u;
            }
        }
        for (uint32_t w = t; w < nclear; w += 256) s_buf[w] = 0u;
        __syncthreads();
        // This thread's count of each digit before each of its keys.  Ranks
        // stay below 2^16 (a sub-chunk holds 6144 keys), so two share a
        // register: fewer live registers, more waves per SIMD.
        uint32_t r2[kItems / 2];
#pragma unroll
        for (int q = 0; q < kItems / 2; ++q) r2[q] = 0u;
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            if (i0 + it < m) {
                const uint32_t d = (k[it] >> shift) & mask;
                const uint32_t e = d * 256u + t;
                const uint32_t h = 16u * (e & 1u);
                const uint32_t old = atomicAdd(&s_buf[cnt_slot(e >> 1)], 1u << h);
                r2[it >> 1] |= ((old >> h) & 0xFFFFu) << (16 * (it & 1));
            }
        }
        __syncthreads();
        // Raking exclusive scan of the counters in (digit, thread) order; the
        // words are read again for the second sweep rather than held.
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < kBins / 2; ++j) {
            if ((uint32_t)j < rake) {
                const uint32_t w = s_buf[cnt_slot(t * rake + j)];
                sum += (w & 0xFFFFu) + (w >> 16);
            }
        }
        uint32_t acc = block_excl_scan(sum, lds, nullptr);
#pragma unroll
        for (int j = 0; j < kBins / 2; ++j) {
            if ((uint32_t)j < rake) {
                const uint32_t w = s_buf[cnt_slot(t * rake + j)];
                const uint32_t e0 = acc;
                acc += w & 0xFFFFu;
                s_buf[cnt_slot(t * rake + j)] = e0 | (acc << 16);
                acc += w >> 16;
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            if (i0 + it < m) {
                const uint32_t e = ((k[it] >> shift) & mask) * 256u + t;
                const uint32_t first = (s_buf[cnt_slot(e >> 1)] >> (16u * (e & 1u))) & 0xFFFFu;
                r2[it >> 1] += first << (16 * (it & 1));  // no carry: every rank is below 2^16
            }
        }
        if (t < bins) dstart[t] = s_buf[cnt_slot(t * 128u)] & 0xFFFFu;
        if (t == 0) dstart[bins] = m;
        __syncthreads();  // every counter read is done before the keys overwrite them
        if (t < bins) {
            gbase[t] = run[t];
            run[t] += dstart[t + 1] - dstart[t];
        }
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            if (i0 + it < m) {
                const uint32_t rk = (r2[it >> 1] >> (16 * (it & 1))) & 0xFFFFu;
                s_keys[rk] = k[it];
                if (has_v) s_vals[rk] = v[it];
            }
        }
        __syncthreads();
        for (uint32_t p = t; p < m; p += 256) {
            const uint32_t kk = s_keys[p];
            const uint32_t d = (kk >> shift) & mask;
            const uint32_t o = gbase[d] + (p - dstart[d]);
            if (o < n) {  // always true for consistent counts; keeps every write in bounds
                kout[o] = kk;
                if (has_v) vout[o] = s_vals[p];
            }
        }
        __syncthreads();
    }
}

template <bool kHasV, int kBits>
__global__ __launch_bounds__(256, (kHasV || kBits > 6) ? 2 : 4) void k_rs_scatter_cnt(const uint32_t* __restrict__ kin,
                                                        const uint32_t* __restrict__ vin,
                                                        uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                        const uint32_t* __restrict__ n_dev, uint32_t n_host,
                                                        int shift, int bits, const uint32_t* __restrict__ counts,
                                                        const uint32_t* __restrict__ totals, RsGate gate) {
    __shared__ uint32_t smem[rs_scatter_cnt_lds<kHasV, kBits>()];
    const uint32_t n = n_dev ? *n_dev : n_host;
    if (n < gate.lo || n > gate.hi) return;
    rs_scatter_cnt_body<kHasV, kBits>(kin, vin, kout, vout, n, shift, bits, counts, totals, gridDim.x, smem);
}

// Either form of a pass on the device count: the small form (1024-key
// sub-chunks, ballot ranks, g_small blocks) up to kRsSplitKeys keys, the
// counter-ranked form (g_big blocks) above.  One launch of max(g_small,
// g_big) blocks each; blocks past the chosen form's grid return.
__global__ __launch_bounds__(256) void k_rs_hist_dual(const uint32_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ n_dev, int shift, int bits,
                                                      uint32_t* __restrict__ counts, uint32_t g_small, uint32_t g_big) {
    __shared__ uint32_t smem[kRsBins];
    const uint32_t n = *n_dev;
    if (n <= kRsSplitKeys) {
        if (blockIdx.x < g_small) rs_hist_body<kRsItemsSmall>(keys, n, shift, bits, counts, g_small, smem);
    } else if (blockIdx.x < g_big) {
        rs_hist_body<kRsItemsBig>(keys, n, shift, bits, counts, g_big, smem);
    }
}

template <bool kHasV, int kBits>
__global__ __launch_bounds__(256, (kHasV || kBits > 6) ? 2 : 4) void k_rs_scatter_dual(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, int shift, int bits,
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals, uint32_t g_small, uint32_t g_big) {
    constexpr int kSmall = rs_scatter_lds<kRsItemsSmall>(), kBig = rs_scatter_cnt_lds<kHasV, kBits>();
    __shared__ uint32_t smem[kSmall > kBig ? kSmall : kBig];
    const uint32_t n = *n_dev;
    if (n <= kRsSplitKeys) {
        if (blockIdx.x < g_small)
            rs_scatter_body<kRsItemsSmall>(kin, vin, kout, kHasV ? vout : nullptr, n, shift, bits, counts, totals,
                                           g_small, smem);
    } else if (blockIdx.x < g_big) {
        rs_scatter_cnt_body<kHasV, kBits>(kin, vin, kout, vout, n, shift, bits, counts, totals, g_big, smem);
    }
}

uint32_t rs_grid(int64_t n_cap, int items) {
    const int64_t g = ceil_div(n_cap > 0 ? n_cap : 1, 256 * items);
    return (uint32_t)(g < kRsGrid ? g : kRsGrid);
}

}  // namespace

size_t radix_tmp_bytes(int64_t n_cap) {
    (void)n_cap;  // the grid, and so the count table, is at most kRsGrid blocks for any size
    return ((size_t)kRsBins * kRsGrid + kRsBins + 64) * sizeof(uint32_t) + 256;
}

hipError_t radix_sort(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, const uint32_t* n_dev,
                      int64_t n_cap, int key_bits, bool iota, void* tmp, hipStream_t s, bool* in_b, int64_t n_hint,
                      int key_shift) {
    *in_b = false;
    if (n_cap <= 0 || key_bits <= 0) return hipSuccess;
    if (n_cap > 0xFFFFFFFFll) return hipErrorInvalidValue;
    // Small sorts (expected keys per block of the full grid below 4096):
    // 1024-key sub-chunks.  An unknown count (n_hint < 0) that may exceed
    // kRsSplitKeys launches both forms, gated on the device count.
    const bool both = n_hint < 0 && n_dev && n_cap > (int64_t)kRsSplitKeys;
    const int64_t n_exp = n_hint > 0 && n_hint < n_cap ? n_hint : n_hint < 0 ? 1 : n_cap;
    const bool small = n_exp <= (int64_t)kRsGrid * 256 * kRsItemsSmall;
    const bool big = both || !small;
    const uint32_t grid_small = kRsSmallGrid, grid_big = rs_grid(n_cap, kRsItemsBig);
    const RsGate g_small = both ? RsGate{0u, kRsSplitKeys} : kRsAlways;
    const RsGate g_big = both ? RsGate{kRsSplitKeys + 1u, 0xFFFFFFFFu} : kRsAlways;
    uint32_t* counts = (uint32_t*)tmp;
    uint32_t* totals = counts + (size_t)kRsBins * kRsGrid;  // past the largest count table
    const int passes = (key_bits + kRsMaxBits - 1) / kRsMaxBits;
    const int per = (key_bits + passes - 1) / passes;
    // The counter-ranked scatter loads 16-byte vectors.
    const auto a16 = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
    const bool aligned = a16(ka) && a16(kb) && a16(va) && a16(vb);
    uint32_t *ki = ka, *ko = kb, *vo = vb;
    const uint32_t* vi = iota ? nullptr : va;
    bool cur_b = false;
    if (key_shift < 0 || key_shift + key_bits > 32) return hipErrorInvalidValue;
    for (int shift = key_shift; shift < key_shift + key_bits; shift += per) {
        const int bits = key_shift + key_bits - shift < per ? key_shift + key_bits - shift : per;
        if (both && bits <= kRsCntMaxBits && aligned) {
            // One launch per kernel, the form chosen by each block from the
            // device count.
            const dim3 gd(grid_small > grid_big ? grid_small : grid_big);
            hipLaunchKernelGGL(k_rs_hist_dual, gd, dim3(256), 0, s, ki, n_dev, shift, bits, counts, grid_small,
                               grid_big);
            hipLaunchKernelGGL(k_rs_scan, dim3(1u << bits), dim3(256), 0, s, counts, grid_small, totals, grid_big,
                               n_dev);
            if (vo && bits <= 6)
                hipLaunchKernelGGL((k_rs_scatter_dual<true, 6>), gd, dim3(256), 0, s, ki, vi, ko, vo, n_dev, shift, bits,
                                   counts, totals, grid_small, grid_big);
            else if (vo)
                hipLaunchKernelGGL((k_rs_scatter_dual<true, 7>), gd, dim3(256), 0, s, ki, vi, ko, vo, n_dev, shift, bits,
                                   counts, totals, grid_small, grid_big);
            else if (bits <= 6)
                hipLaunchKernelGGL((k_rs_scatter_dual<false, 6>), gd, dim3(256), 0, s, ki, vi, ko, vo, n_dev, shift,
                                   bits, counts, totals, grid_small, grid_big);
            else
                hipLaunchKernelGGL((k_rs_scatter_dual<false, 7>), gd, dim3(256), 0, s, ki, vi, ko, vo, n_dev, shift,
                                   bits, counts, totals, grid_small, grid_big);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            cur_b = !cur_b;
            if (cur_b) {
                ki = kb; vi = vb; ko = ka; vo = va;
            } else {
                ki = ka; vi = va; ko = kb; vo = vb;
            }
            continue;
        }
        if (small)
            hipLaunchKernelGGL(k_rs_hist<kRsItemsSmall>, dim3(grid_small), dim3(256), 0, s, ki, n_dev,
                               (uint32_t)n_cap, shift, bits, counts, g_small);
        if (big)
            hipLaunchKernelGGL(k_rs_hist<kRsItemsBig>, dim3(grid_big), dim3(256), 0, s, ki, n_dev, (uint32_t)n_cap,
                               shift, bits, counts, g_big);
        hipLaunchKernelGGL(k_rs_scan, dim3(1u << bits), dim3(256), 0, s, counts, small ? grid_small : grid_big, totals,
                           grid_big, both ? n_dev : nullptr);
        if (small)
            hipLaunchKernelGGL(k_rs_scatter<kRsItemsSmall>, dim3(grid_small), dim3(256), 0, s, ki, vi, ko, vo, n_dev,
                               (uint32_t)n_cap, shift, bits, counts, totals, g_small);
        if (!big) {
        } else if (bits <= 6 && aligned && vo) {
            hipLaunchKernelGGL((k_rs_scatter_cnt<true, 6>), dim3(grid_big), dim3(256), 0, s, ki, vi, ko, vo, n_dev,
                               (uint32_t)n_cap, shift, bits, counts, totals, g_big);
        } else if (bits <= 6 && aligned) {
            hipLaunchKernelGGL((k_rs_scatter_cnt<false, 6>), dim3(grid_big), dim3(256), 0, s, ki, vi, ko, vo, n_dev,
                               (uint32_t)n_cap, shift, bits, counts, totals, g_big);
        } else if (bits <= kRsCntMaxBits && aligned && vo) {
            hipLaunchKernelGGL((k_rs_scatter_cnt<true, 7>), dim3(grid_big), dim3(256), 0, s, ki, vi, ko, vo, n_dev,
                               (uint32_t)n_cap, shift, bits, counts, totals, g_big);
        } else if (bits <= kRsCntMaxBits && aligned) {
            hipLaunchKernelGGL((k_rs_scatter_cnt<false, 7>), dim3(grid_big), dim3(256), 0, s, ki, vi, ko, vo, n_dev,
                               (uint32_t)n_cap, shift, bits, counts, totals, g_big);
        } else {
            hipLaunchKernelGGL(k_rs_scatter<kRsItemsBig>, dim3(grid_big), dim3(256), 0, s, ki, vi, ko, vo, n_dev,
                               (uint32_t)n_cap, shift, bits, counts, totals, g_big);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur_b = !cur_b;
        if (cur_b) {
            ki = kb; vi = vb; ko = ka; vo = va;
        } else {
            ki = ka; vi = va; ko = kb; vo = vb;
        }
    }
    *in_b = cur_b;
    return hipSuccess;
}

}  // namespace bgs
