// Device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// Radix sort: reduce-then-scan per 8-bit digit.  Each pass is three steps:
// per-block digit histograms (LDS), an exclusive scan of the digit-major
// histogram matrix, and a scatter in which every block ranks its 4096 keys
// stably with wave64 ballots (match-any on the digit), reorders them in LDS
// and writes digit runs out contiguously.  No inter-block waiting: blocks
// never spin on each other.
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

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

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
        hipError_t e = hipMemsetAsync(partials, 0, sizeof(uint32_t), s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(256), 0, s, in, idx, n_dev, n_cap, partials, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Radix sort
// ---------------------------------------------------------------------------
namespace {

// Lanes of the wave whose 8-bit digit equals this lane's (among `valid`).
__device__ inline uint64_t match_digit(uint32_t d, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t bal = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return peers;
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ n_dev, uint32_t n_host, int shift,
                                                    uint32_t mask, uint32_t* __restrict__ hist, uint32_t nb) {
    __shared__ uint32_t h[256];
    const uint32_t n = n_dev ? *n_dev : n_host;
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixBlock;
    if (base < n) {
        const uint32_t lane = lane_id();
        const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll 4
        for (int j = 0; j < kRadixItems; ++j) {
            uint64_t i = base + (uint64_t)j * 256 + threadIdx.x;
            bool ok = i < n;
            uint32_t d = ok ? (keys[i] >> shift) & mask : 0u;
            uint64_t peers = match_digit(d, __ballot(ok));
            if (ok && (peers & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       const uint32_t* __restrict__ n_dev, uint32_t n_host,
                                                       int shift, uint32_t mask,
                                                       const uint32_t* __restrict__ offs, uint32_t nb) {
    __shared__ uint32_t s_keys[kRadixBlock];
    __shared__ uint32_t s_vals[kRadixBlock];
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t lds[4];
    const uint32_t n = n_dev ? *n_dev : n_host;
    const uint64_t base = (uint64_t)blockIdx.x * kRadixBlock;
    if (base >= n) return;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int w = 0; w < 4; ++w) cnt[w][threadIdx.x] = 0;
    __syncthreads();

    // Stable rank of every key within its wave's 1024-key segment: the
    // segment is walked in 16 steps of 64 consecutive keys; lanes with the
    // same digit are found with ballots and the wave's running per-digit
    // count lives in LDS.
    uint32_t k[kRadixItems], v[kRadixItems], r[kRadixItems];
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        uint64_t i = base + (uint64_t)wave * (64 * kRadixItems) + (uint64_t)it * 64 + lane;
        bool ok = i < n;
        k[it] = ok ? kin[i] : 0xFFFFFFFFu;
        v[it] = ok ? (vin ? vin[i] : (uint32_t)i) : 0u;
        uint32_t d = (k[it] >> shift) & mask;
        uint64_t valid = __ballot(ok);
        uint64_t peers = match_digit(d, valid);
        uint32_t c = ok ? cnt[wave][d] : 0u;
        r[it] = c + (uint32_t)__popcll(peers & lt);
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & lt) == 0) cnt[wave][d] = c + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (!ok) r[it] = 0xFFFFFFFFu;
    }
    __syncthreads();
    {
        const uint32_t d = threadIdx.x;
        uint32_t c0 = cnt[0][d], c1 = cnt[1][d], c2 = cnt[2][d], c3 = cnt[3][d];
        uint32_t tot = c0 + c1 + c2 + c3;
        uint32_t st = block_excl_scan(tot, lds, nullptr);
        cnt[0][d] = st;
        cnt[1][d] = st + c0;
        cnt[2][d] = st + c0 + c1;
        cnt[3][d] = st + c0 + c1 + c2;
        dstart[d] = st;
        gbase[d] = offs[(uint64_t)d * nb + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        if (r[it] != 0xFFFFFFFFu) {
            uint32_t d = (k[it] >> shift) & mask;
            uint32_t pos = cnt[wave][d] + r[it];
            s_keys[pos] = k[it];
            s_vals[pos] = v[it];
        }
    }
    __syncthreads();
    const uint32_t m = (uint32_t)min<uint64_t>((uint64_t)kRadixBlock, (uint64_t)n - base);
    for (uint32_t p = threadIdx.x; p < m; p += 256) {
        uint32_t kk = s_keys[p];
        uint32_t d = (kk >> shift) & mask;
        uint32_t o = gbase[d] + (p - dstart[d]);
        if (o < n) {
            kout[o] = kk;
            vout[o] = s_vals[p];
        }
    }
}

}  // namespace

size_t radix_tmp_bytes(int64_t n_cap) {
    int64_t nb = ceil_div(n_cap > 0 ? n_cap : 1, kRadixBlock);
    size_t hist = (size_t)256 * nb;
    size_t tmp = scan_tmp_elems((int64_t)hist);
    return (hist + 64 + tmp) * sizeof(uint32_t) + 256;
}

hipError_t radix_sort(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, const uint32_t* n_dev,
                      int64_t n_cap, int key_bits, bool iota, void* tmp, hipStream_t s, bool* in_b) {
    *in_b = false;
    if (n_cap <= 0 || key_bits <= 0) return hipSuccess;
    const int64_t nb = ceil_div(n_cap, kRadixBlock);
    uint32_t* hist = (uint32_t*)tmp;
    uint32_t* stmp = hist + 256 * nb + 64;
    uint32_t *ki = ka, *ko = kb, *vo = vb;
    const uint32_t* vi = iota ? nullptr : va;
    bool cur_b = false;
    for (int shift = 0; shift < key_bits; shift += 8) {
        int bits = key_bits - shift < 8 ? key_bits - shift : 8;
        uint32_t mask = (1u << bits) - 1u;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(256), 0, s, ki, n_dev, (uint32_t)n_cap, shift,
                           mask, hist, (uint32_t)nb);
        hipError_t e = exclusive_scan(hist, nullptr, hist, nullptr, 256 * nb, stmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(256), 0, s, ki, vi, ko, vo, n_dev,
                           (uint32_t)n_cap, shift, mask, hist, (uint32_t)nb);
        e = hipGetLastError();
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
