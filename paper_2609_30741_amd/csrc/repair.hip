// Learned gap/edge repair network: inference and training kernels.
//
// 3x3 convolutions run as implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, fp32 accumulate).  Forward: rows of the GEMM
// are output channels (weights packed [cout padded to 16][9][cin padded to
// 16], each row padded with zeros to a multiple of 32), columns are 16
// consecutive pixels of one image row, the reduction runs over (tap, input
// channel).  The input-gradient pass is the same kernel
// with the weights transposed and flipped.  The weight gradient is a GEMM
// over pixels: each block accumulates a slab of rows into per-block
// partials that a second kernel adds in a fixed order, so results are
// deterministic.  Activations and gradients between layers are stored as
// bf16 [B][H][W][C], channels innermost; a layer may read or write a
// channel slice of a larger tensor (the pixel stride exceeds the slice),
// which is how the skip connections land in the decoder's concatenated
// inputs without copies.  The images the network reads and writes are
// planar fp32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>

#include "bgs_repair.h"

namespace {

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct LayerDef {
    int cin, cout, relu;
};
// e1a e1b e2a e2b e3a e3b d2 d1 out
constexpr int kLayers = 9;
constexpr LayerDef kNet[kLayers] = {{5, 16, 1},  {16, 16, 1}, {16, 32, 1}, {32, 32, 1}, {32, 64, 1},
                                    {64, 64, 1}, {96, 32, 1}, {48, 16, 1}, {16, 4, 0}};
enum { E1A, E1B, E2A, E2B, E3A, E3B, D2, D1, OUT };

constexpr int pad16(int v) { return (v + 15) & ~15; }

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    // Round to nearest even (values are finite).
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// Convolution (forward, or input gradient with transposed weights).
// Activations and gradients are bf16 [B][H][W][C] with the channels of a
// pixel contiguous; a tensor's pixel stride (ps) is a multiple of 8 and may
// exceed the channels a layer reads or writes (a slice of a concatenation,
// or zero padding), and every buffer is 16-byte aligned.
// ---------------------------------------------------------------------------
struct ConvArgs {
    const uint16_t* in;  // channel 0 of the input
    int64_t in_bs;       // elements per image
    int in_ps;           // elements per pixel
    int cin;
    // Optional half-resolution source of input channels [0, up_c): read at
    // (y / 2, x / 2), the nearest 2x upsample, so a decoder's concatenated
    // input needs no upsampled copy.  Channel ci >= up_c is channel
    // ci - up_c of in.
    const uint16_t* up;
    int64_t up_bs;
    int up_ps;
    int up_c;
    const uint16_t* w;  // [pad16(cout)][kpad] bf16, k = tap * cpad + ci, zero for k >= 9 cpad
    int kpad;           // pad32(9 cpad)
    const float* bias;  // may be null
    int cout;           // a multiple of 4
    uint16_t* out;      // channel 0 of the output (bf16, out_bs, out_ps), or
    float* out_f;       // fp32 [B][cout][H][W] planes (exactly one is set)
    int64_t out_bs;
    int out_ps;
    const uint16_t* mask;  // may be null: output zero where mask <= 0 (layout of out)
    int64_t mask_bs;
    int mask_ps;
    // May be null: also store the 2x2 mean of the (bf16) output, [H/2][W/2]
    // pixels of pool_ps elements (H and W even).
    uint16_t* pool;
    int64_t pool_bs;
    int pool_ps;
    int relu;
    int H, W;
};

// Block: 4 waves over 64 pixels (x from blockIdx.x * 64) of R consecutive
// rows from R blockIdx.y; blockIdx.z = image * groups + group, a group
// being MT <= 4 16-row tiles of output channels.
// The block first stages input rows R blockIdx.y - 1 .. + R, x from
// blockIdx.x * 64 - 1 to + 64 (zero outside the image), of every input
// channel (padded to CPAD, a multiple of 16, with zeros) in LDS:
// [R + 2][66][CPAD + conv_pad(CPAD)] bf16, one 16-byte load and store per
// 8 channels of a pixel.  The reduction index is k = tap * CPAD + ci in
// 32-deep slices of v_mfma_f32_16x16x32_bf16; a lane's eight operands of a
// slice are eight consecutive channels of one tap, one 16-byte LDS read,
// and each weight operand serves all R rows and all of a wave's column
// tiles.
constexpr int kConvCols = 66;

constexpr int pad32(int v) { return (v + 31) & ~31; }
// Spare channel slots per staged pixel, by width, chosen by measurement
// over 0 to 32 spare slots (LDS bank-conflict counter and kernel time): the
// 16-byte operand reads of 48 and 96 channels are cheapest with none (and
// the smaller stage fits more blocks per CU: 96 channels at 800x600, 29 ->
// 23 us), those of 32 and 64 channels with 16, and 16 channels run
// fastest with 8.
constexpr int conv_pad(int cpad) { return cpad == 16 ? 8 : cpad == 32 || cpad == 64 ? 16 : 0; }
constexpr size_t conv_lds_bytes(int cpad, int rows) {
    return (size_t)(rows + 2) * kConvCols * (cpad + conv_pad(cpad)) * sizeof(uint16_t);
}

template <int CPAD, int MT, int R>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a) {
    constexpr int PS = CPAD + conv_pad(CPAD);  // staged bf16 per pixel
    constexpr int G = CPAD / 8;               // 16-byte channel groups per pixel
    constexpr int SL = pad32(9 * CPAD) / 32;  // reduction slices
    extern __shared__ uint4 s_raw[];
    uint16_t* s_in = reinterpret_cast<uint16_t*>(s_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int groups = (a.cout + 16 * MT - 1) / (16 * MT);
    const int y0 = blockIdx.y * R, b = blockIdx.z / groups, m0 = (blockIdx.z - b * groups) * MT;
    const int xb = blockIdx.x * 64;
    const int W2 = a.W >> 1;
    const uint16_t* inb = a.in + (int64_t)b * a.in_bs;
    const uint16_t* upb = a.up ? a.up + (int64_t)b * a.up_bs : nullptr;
    const int n = lane & 15, kg = lane >> 4;
    const int mt = min(MT, ((a.cout + 15) >> 4) - m0);
    // Wave w computes output tile m = w % MT (of the group) for CT = 4 / CW
    // consecutive 16-pixel column tiles from column tile CT (w / MT), so a
    // block reads each weight row 4 / MT times instead of 4 (MT = 3: waves
    // 0-2 take all four column tiles, wave 3 only helps with the fill).
    constexpr int CW = MT == 1 ? 4 : MT == 2 ? 2 : 1;  // waves per tile
    constexpr int CT = 4 / CW;
    const int wm = wave % MT, wc = (wave / MT) * CT;
    const bool busy = wave < MT * CW;
    // Weight operands run P slices ahead of their use in a register ring;
    // the first P are in flight during the fill.
    constexpr int P = SL < 8 ? SL : 8;
    const uint16_t* wl = a.w + (size_t)((m0 + min(wm, mt - 1)) * 16 + n) * a.kpad + 8 * kg;
    uint4 wq[P];
#pragma unroll
    for (int s = 0; s < P; ++s) wq[s] = *reinterpret_cast<const uint4*>(wl + 32 * s);
    // Fill: item = (row, column, channel group), group fastest, so a wave's
    // loads walk consecutive 16-byte words of consecutive pixels.  Up to 12
    // items' loads per thread are in flight before their stores (one round
    // trip for all but the widest input).  Channels at or past
    // cin read as zero (a group past cin is not loaded: it may lie beyond
    // the tensor's pixel stride).
    constexpr int items = (R + 2) * kConvCols * G;
    constexpr int U = (items + 255) / 256 < 12 ? (items + 255) / 256 : 12;
    for (int i0 = threadIdx.x; i0 < items; i0 += 256 * U) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int it = i0 + 256 * u;
            const int g = it % G, rc = it / G;
            const int c = rc % kConvCols, r = rc / kConvCols;
            const int yy = y0 + r - 1, xx = xb + c - 1, ci = 8 * g;
            const bool ok = it < items && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W && ci < a.cin;
            v[u] = uint4{0u, 0u, 0u, 0u};
            if (ok) {
                const uint16_t* src = ci < a.up_c
                                          ? upb + ((int64_t)(yy >> 1) * W2 + (xx >> 1)) * a.up_ps + ci
                                          : inb + ((int64_t)yy * a.W + xx) * a.in_ps + (ci - a.up_c);
                v[u] = *reinterpret_cast<const uint4*>(src);
                const int left = a.cin - ci;  // channels of this group that exist
                if (left < 8) {
                    uint32_t* q = reinterpret_cast<uint32_t*>(&v[u]);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t keep = (2 * k + 1 < left ? 0xFFFF0000u : 0u) | (2 * k < left ? 0xFFFFu : 0u);
                        q[k] &= keep;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int it = i0 + 256 * u;
            if (it < items) {
                const int g = it % G, rc = it / G;
                *reinterpret_cast<uint4*>(s_in + rc * PS + 8 * g) = v[u];
            }
        }
    }
    __syncthreads();
    if (!busy || wm >= mt || xb + 16 * wc >= a.W) return;  // whole wave, after the block's only barrier
    v4f acc[CT][R];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[c][r] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < SL; ++s) {
        // This lane's operands: k = 32 s + 8 kg .. + 7, one tap t and eight
        // channels from ci.  Past the last tap (the zero padding of the
        // reduction) the operands are zero.
        const int k = 32 * s + 8 * kg;
        const int t = k / CPAD, ci = k - t * CPAD;
        const int ty = t / 3, tx = t - 3 * ty;
        const v8bf av = __builtin_bit_cast(v8bf, wq[s % P]);
        if (s + P < SL) wq[s % P] = *reinterpret_cast<const uint4*>(wl + 32 * (s + P));
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int col = 16 * (wc + c) + n;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                uint4 q = uint4{0u, 0u, 0u, 0u};
                if (32 * s + 32 <= 9 * CPAD || t < 9)
                    q = *reinterpret_cast<const uint4*>(s_in + ((r + ty) * kConvCols + col + tx) * PS + ci);
                acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(v8bf, q), acc[c][r], 0, 0, 0);
            }
        }
    }
    // Lane holds output channels co .. co + 3 of pixel column n of each
    // column tile: one 8-byte store per row and tile (cout is a multiple of 4).
    const int co = (m0 + wm) * 16 + 4 * kg;
    if (co >= a.cout) return;
    float bias[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[j] = a.bias ? a.bias[co + j] : 0.f;
    float st[CT][R][4];  // the stored values, for the pool
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int x = xb + 16 * (wc + c) + n;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = y0 + r;
            const bool in = x < a.W && y < a.H;
            const int64_t pix = (int64_t)y * a.W + x;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = acc[c][r][j] + bias[j];
                if (a.relu) v[j] = fmaxf(v[j], 0.f);
            }
            if (in && a.mask) {
                const uint2 mk =
                    *reinterpret_cast<const uint2*>(a.mask + (int64_t)b * a.mask_bs + pix * a.mask_ps + co);
                if (!(bf2f((uint16_t)(mk.x & 0xFFFFu)) > 0.f)) v[0] = 0.f;
                if (!(bf2f((uint16_t)(mk.x >> 16)) > 0.f)) v[1] = 0.f;
                if (!(bf2f((uint16_t)(mk.y & 0xFFFFu)) > 0.f)) v[2] = 0.f;
                if (!(bf2f((uint16_t)(mk.y >> 16)) > 0.f)) v[3] = 0.f;
            }
            uint16_t h[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                h[j] = f2bf(v[j]);
                st[c][r][j] = bf2f(h[j]);
            }
            if (!in) continue;
            if (a.out_f) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    a.out_f[(int64_t)b * a.out_bs + (int64_t)(co + j) * a.H * a.W + pix] = v[j];
            } else {
                *reinterpret_cast<uint2*>(a.out + (int64_t)b * a.out_bs + pix * a.out_ps + co) =
                    uint2{(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16)};
            }
        }
    }
    if (!a.pool) return;
    // 2x2 mean of the stored values: rows r and r + 1 of the lane (R and the
    // block's first row are even), columns of lanes n and n ^ 1 (same kg),
    // summed in the order (x, y), (x + 1, y), (x, y + 1), (x + 1, y + 1).
    // With W and H even a pair of columns or rows is inside the image or
    // outside together.
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int x = xb + 16 * (wc + c) + n;
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            const int y = y0 + r;
            float q[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float s0 = st[c][r][j], s2 = st[c][r + 1][j];
                const float s1 = __shfl_xor(s0, 1, 64), s3 = __shfl_xor(s2, 1, 64);
                q[j] = 0.25f * (((s0 + s1) + s2) + s3);
            }
            if ((n & 1) || x >= a.W || y >= a.H) continue;
            const int64_t pp = (int64_t)(y >> 1) * (a.W >> 1) + (x >> 1);
            *reinterpret_cast<uint2*>(a.pool + (int64_t)b * a.pool_bs + pp * a.pool_ps + co) =
                uint2{(uint32_t)f2bf(q[0]) | ((uint32_t)f2bf(q[1]) << 16),
                      (uint32_t)f2bf(q[2]) | ((uint32_t)f2bf(q[3]) << 16)};
        }
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradient: part[chunk][co][col] = sum over the chunk's
// pixels of g[p, co] * in[p + tap offset, ci] for col = ci * 9 + tap < K,
// and of g[p, co] (a column of ones) for col = K, the bias.  Block: 4
// waves, one 16-column tile each; blockIdx.y: chunk of image rows.  The
// reduction runs over 32 pixels of a row per v_mfma_f32_16x16x32_bf16.
// ---------------------------------------------------------------------------
struct WgradArgs {
    const uint16_t* g;  // layer output gradient, [B][H][W] pixels of g_ps elements
    int64_t g_bs;
    int g_ps;
    int cout;
    const uint16_t* in;  // layer input, in_ps elements per pixel
    int64_t in_bs;
    int in_ps;
    int cin;
    int B, H, W;
    int rows;  // image rows (over the whole batch) per chunk
    float* part;
};

__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int K = a.cin * 9, KC = K + 1;
    const int nt = blockIdx.x * 4 + wave;
    if (nt * 16 >= KC) return;  // whole wave
    const int n = lane & 15, kq = (lane >> 4) * 8;
    const int col = nt * 16 + n;
    const bool col_ok = col < K, is_bias = col == K;
    const int ci = col_ok ? col / 9 : 0, t = col_ok ? col - ci * 9 : 4;
    const int ky = t / 3, kx = t - ky * 3;
    const int mt = (a.cout + 15) >> 4;
    v4f acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
    const int r0 = blockIdx.y * a.rows, r1 = min(r0 + a.rows, a.B * a.H);
    for (int r = r0; r < r1; ++r) {
        const int b = r / a.H, y = r - b * a.H;
        const uint16_t* gb = a.g + (int64_t)b * a.g_bs + (int64_t)y * a.W * a.g_ps;
        const uint16_t* ib = a.in + (int64_t)b * a.in_bs + ci;
        const int yy = y + ky - 1;
        const bool row_ok = col_ok && yy >= 0 && yy < a.H;
#pragma unroll 2
        for (int xb = 0; xb < a.W; xb += 32) {
            v8s bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int xp = xb + kq + j, xx = xp + kx - 1;
                const bool ok = row_ok && xp < a.W && xx >= 0 && xx < a.W;
                bv[j] = (short)(ok ? ib[((int64_t)yy * a.W + xx) * a.in_ps]
                                   : (is_bias && xp < a.W) ? (uint16_t)0x3F80u : (uint16_t)0);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (m < mt) {
                    const int co = m * 16 + n;
                    v8s av;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const int xp = xb + kq + j;
                        av[j] = (short)((co < a.cout && xp < a.W) ? gb[(int64_t)xp * a.g_ps + co] : (uint16_t)0);
                    }
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av),
                                                                    __builtin_bit_cast(v8bf, bv), acc[m], 0, 0, 0);
                }
            }
        }
    }
    if (col >= KC) return;
    float* pb = a.part + (size_t)blockIdx.y * a.cout * KC;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (m >= mt) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = m * 16 + (lane >> 4) * 4 + j;
            if (co < a.cout) pb[(size_t)co * KC + col] = acc[m][j];
        }
    }
}

// grad (the layer's W[cout][K] then b[cout]) from the partials in a fixed
// order: block of 64 outputs; wave q adds the q-th quarter of the chunks in
// chunk order, then ((q0 + q1) + (q2 + q3)).
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int chunks, int cout, int K,
                                                      float* __restrict__ grad) {
    __shared__ float s_q[4][64];
    const int KC = K + 1;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int per = (chunks + 3) / 4, c0 = q * per, c1 = min(chunks, c0 + per);
    float s = 0.f;
    if (i < cout * KC)
        for (int c = c0; c < c1; ++c) s += part[(size_t)c * cout * KC + i];
    s_q[q][lane] = s;
    __syncthreads();
    if (q != 0 || i >= cout * KC) return;
    const float v = (s_q[0][lane] + s_q[1][lane]) + (s_q[2][lane] + s_q[3][lane]);
    const int co = i / KC, col = i - co * KC;
    grad[col < K ? co * K + col : cout * K + co] = v;
}

__device__ __forceinline__ float block_sum(float v, float* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const float s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// Weight packing (fp32 master -> bf16 GEMM operands), pooling, upsampling,
// gradient merges, input assembly, output and loss.
// ---------------------------------------------------------------------------
// Column k = tap * cpad + c of a packed row of kpad columns (zero from
// 9 cpad on).  Forward: row = output channel, c = input channel,
// W[row][c][tap].  Transposed (input gradient): row = input channel, c =
// output channel, W[c][row][8 - tap] (the kernel flipped).  One launch
// packs every job: job j covers elements [start[j], start[j + 1]) of the
// grid.
struct PackJob {
    const float* w;
    uint16_t* out;
    int cin, cout, transpose, cpad, kpad;
};
struct PackJobs {
    PackJob job[2 * kLayers];
    int start[2 * kLayers + 1];
    int n;
};

__global__ __launch_bounds__(256) void k_pack(PackJobs J) {
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= J.start[J.n]) return;
    int jb = 0;
    while (g >= J.start[jb + 1]) ++jb;
    const PackJob& P = J.job[jb];
    const float* __restrict__ w = P.w;
    const int cin = P.cin, cout = P.cout, transpose = P.transpose, cpad = P.cpad, kpad = P.kpad;
    const int i = g - J.start[jb];
    const int m = i / kpad, k = i - m * kpad;
    const int t = k / cpad, c = k - t * cpad;
    float v = 0.f;
    if (t < 9) {
        if (!transpose) {
            if (m < cout && c < cin) v = w[(m * cin + c) * 9 + t];
        } else {
            if (m < cin && c < cout) v = w[(c * cin + m) * 9 + (8 - t)];
        }
    }
    P.out[i] = f2bf(v);
}

// The channel kernels below take one pixel's eight channels (one 16-byte
// word) per thread: grid over B * pixels * C / 8 (C a multiple of 8),
// channel group fastest.
__device__ __forceinline__ void unpack8(uint4 q, float* f) {
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = bf2f((uint16_t)(w[k] & 0xFFFFu));
        f[2 * k + 1] = bf2f((uint16_t)(w[k] >> 16));
    }
}
__device__ __forceinline__ uint4 pack8(const float* f) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(f[2 * k]) | ((uint32_t)f2bf(f[2 * k + 1]) << 16);
    return uint4{w[0], w[1], w[2], w[3]};
}
__device__ __forceinline__ uint4 ld8(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ void st8(uint16_t* p, uint4 v) { *reinterpret_cast<uint4*>(p) = v; }

// Index of this thread's (image, pixel, channel group) over n pixels per
// image; false past the end.
__device__ __forceinline__ bool item(int64_t B, int64_t n, int C, int64_t& b, int64_t& p, int& c) {
    const int G = C >> 3;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= B * n * G) return false;
    const int64_t bp = i / G;
    c = (int)(i - bp * G) * 8;
    b = bp / n;
    p = bp - b * n;
    return true;
}

// Nearest 2x upsample of [B][h][w][C] into the first C channel slots of a
// larger tensor (out_bs, out_ps).
__global__ __launch_bounds__(256) void k_up(const uint16_t* __restrict__ in, int B, int C, int h, int w,
                                            uint16_t* __restrict__ out, int64_t out_bs, int out_ps) {
    const int H = 2 * h, W = 2 * w;
    int64_t b, p;
    int c;
    if (!item(B, (int64_t)H * W, C, b, p, c)) return;
    const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
    st8(out + b * out_bs + p * out_ps + c, ld8(in + (b * h * w + (int64_t)(y >> 1) * w + (x >> 1)) * C + c));
}

// Gradient of the upsample: sum of each 2x2 block of the first C channels
// of g (g_bs, g_ps), masked by the activation act [B][H/2][W/2][C] (ReLU
// derivative), into out of that layout.
__global__ __launch_bounds__(256) void k_up_grad(const uint16_t* __restrict__ g, int64_t g_bs, int g_ps, int B, int C,
                                                 int H, int W, const uint16_t* __restrict__ act,
                                                 uint16_t* __restrict__ out) {
    const int h = H / 2, w = W / 2;
    int64_t b, p;
    int c;
    if (!item(B, (int64_t)h * w, C, b, p, c)) return;
    const int Y = (int)(p / w), X = (int)(p - (int64_t)Y * w);
    const uint16_t* q = g + b * g_bs + ((int64_t)(2 * Y) * W + 2 * X) * g_ps + c;
    float f0[8], f1[8], f2[8], f3[8], a[8], o[8];
    unpack8(ld8(q), f0);
    unpack8(ld8(q + g_ps), f1);
    unpack8(ld8(q + (int64_t)W * g_ps), f2);
    unpack8(ld8(q + (int64_t)(W + 1) * g_ps), f3);
    const int64_t oi = (b * h * w + p) * C + c;
    unpack8(ld8(act + oi), a);
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = a[k] > 0.f ? ((f0[k] + f1[k]) + f2[k]) + f3[k] : 0.f;
    st8(out + oi, pack8(o));
}

// Gradient reaching an encoder activation from its skip connection (C
// channels of skip, at skip_bs, skip_ps) and from the pool below it (pg,
// [B][H/2][W/2][C]), masked by the activation (act_bs, act_ps), into out
// [B][H][W][C].
__global__ __launch_bounds__(256) void k_merge(const uint16_t* __restrict__ skip, int64_t skip_bs, int skip_ps,
                                               const uint16_t* __restrict__ pg, const uint16_t* __restrict__ act,
                                               int64_t act_bs, int act_ps, int B, int C, int H, int W,
                                               uint16_t* __restrict__ out) {
    int64_t b, p;
    int c;
    if (!item(B, (int64_t)H * W, C, b, p, c)) return;
    const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
    float sk[8], pl[8], a[8], o[8];
    unpack8(ld8(skip + b * skip_bs + p * skip_ps + c), sk);
    unpack8(ld8(pg + (b * (H / 2) * (W / 2) + (int64_t)(y >> 1) * (W / 2) + (x >> 1)) * C + c), pl);
    unpack8(ld8(act + b * act_bs + p * act_ps + c), a);
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = a[k] > 0.f ? sk[k] + 0.25f * pl[k] : 0.f;
    st8(out + (b * H * W + p) * C + c, pack8(o));
}

// Network input x0 [B][H][W][8]: warped rgb (zero at holes), hole flag,
// 1/z (zero at holes and background), three zero slots.
__global__ __launch_bounds__(256) void k_input(const float* __restrict__ rgb, const float* __restrict__ z,
                                               const uint8_t* __restrict__ hole, int B, int HW,
                                               uint16_t* __restrict__ x0) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)B * HW) return;
    const int64_t b = i / HW, p = i - b * HW;
    const bool h = hole[i] != 0;
    const float zz = z[i];
    float f[8];
#pragma unroll
    for (int c = 0; c < 3; ++c) f[c] = h ? 0.f : rgb[(b * 3 + c) * HW + p];
    f[3] = h ? 1.f : 0.f;
    f[4] = (h || !(zz < INFINITY)) ? 0.f : 1.f / zz;
    f[5] = f[6] = f[7] = 0.f;
    st8(x0 + i * 8, pack8(f));
}

// r: [B][4][HW], channels 0-2 the residual, 3 the predicted squared error.
__global__ __launch_bounds__(256) void k_output(const float* __restrict__ rgb, const uint8_t* __restrict__ hole,
                                                const float* __restrict__ r, int B, int HW,
                                                float* __restrict__ out, float* __restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)B * HW) return;
    const int64_t b = i / HW, p = i - b * HW;
    const bool h = hole[i] != 0;
    const float* rb = r + b * 4 * HW + p;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int64_t q = (b * 3 + c) * HW + p;
        out[q] = h ? rgb[q] + rb[(int64_t)c * HW] : rgb[q];
    }
    if (err) err[i] = h ? rb[3 * (int64_t)HW] : 0.f;
}

// Per-block hole counts.
__global__ __launch_bounds__(256) void k_count(const uint8_t* __restrict__ hole, int64_t n, float* __restrict__ part) {
    __shared__ float red[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const float c = (i < n && hole[i]) ? 1.f : 0.f;
    const float s = block_sum(c, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Predicted error of each image over its holes, first step: block b of
// image y sums err and counts holes over its grid-stride pixels, into
// part[2 (y * kErrParts + b) + {0, 1}].
constexpr int kErrParts = 256;
__global__ __launch_bounds__(256) void k_err_part(const float* __restrict__ err, const uint8_t* __restrict__ hole,
                                                  int64_t HW, float* __restrict__ part) {
    __shared__ float red[4];
    const int64_t img = blockIdx.y;
    float e = 0.f, c = 0.f;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < HW; p += (int64_t)kErrParts * 256) {
        if (hole[img * HW + p]) {
            e += err[img * HW + p];
            c += 1.f;
        }
    }
    e = block_sum(e, red);
    __syncthreads();
    c = block_sum(c, red);
    if (threadIdx.x == 0) {
        part[2 * (img * kErrParts + blockIdx.x)] = e;
        part[2 * (img * kErrParts + blockIdx.x) + 1] = c;
    }
}

// Second step, one block per image: out[y] = sum e / max(1, holes).
__global__ __launch_bounds__(256) void k_err_mean(const float* __restrict__ part, float* __restrict__ out) {
    __shared__ float red[4];
    const int64_t img = blockIdx.x;
    const float* q = part + 2 * img * kErrParts;
    float e = block_sum(q[2 * threadIdx.x], red);
    __syncthreads();
    const float c = block_sum(q[2 * threadIdx.x + 1], red);
    if (threadIdx.x == 0) out[img] = e / fmaxf(c, 1.f);
}

// One block: out[0] = scale * sum of part[0, n) (fixed order per thread,
// then the block tree).
__global__ __launch_bounds__(256) void k_sum(const float* __restrict__ part, int n, const float* __restrict__ div,
                                             float* __restrict__ out) {
    __shared__ float red[4];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = div ? s / (3.f * fmaxf(div[0], 1.f)) : s;
}

// Loss terms per hole pixel: sum over channels of (pred - target)^2 plus
// 3 (e - s)^2, s the pixel's mean squared error (held constant); per-block
// partial sums (k_sum divides by 3 holes).  Gradient with respect to the
// output layer (bf16 [B][H][W][8], slots 4-7 zero): 2 d_c / (3 N) for the
// residual, 2 (e - s) / N for e.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ rgb, const uint8_t* __restrict__ hole,
                                              const float* __restrict__ r, const float* __restrict__ target,
                                              const float* __restrict__ n_hole, int B, int HW,
                                              float* __restrict__ rgb_out, uint16_t* __restrict__ g_r,
                                              float* __restrict__ part) {
    __shared__ float red[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float e = 0.f;
    if (i < (int64_t)B * HW) {
        const int64_t b = i / HW, p = i - b * HW;
        const bool h = hole[i] != 0;
        const float nh = fmaxf(n_hole[0], 1.f);
        const float* rb = r + b * 4 * HW + p;
        float d[3], s2 = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t q = (b * 3 + c) * HW + p;
            const float pred = h ? rgb[q] + rb[(int64_t)c * HW] : rgb[q];
            d[c] = h ? pred - target[q] : 0.f;
            s2 += d[c] * d[c];
            if (rgb_out) rgb_out[q] = pred;
        }
        const float de = h ? rb[3 * (int64_t)HW] - s2 / 3.f : 0.f;
        float gr[8];
#pragma unroll
        for (int c = 0; c < 3; ++c) gr[c] = 2.f * d[c] / (3.f * nh);
        gr[3] = 2.f * de / nh;
        gr[4] = gr[5] = gr[6] = gr[7] = 0.f;
        st8(g_r + i * 8, pack8(gr));
        e = s2 + 3.f * de * de;
    }
    const float sum = block_sum(e, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Host side: parameter offsets, workspace layout, launch sequences.
// ---------------------------------------------------------------------------
int64_t param_offset(int l) {
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += (int64_t)kNet[i].cout * kNet[i].cin * 9 + kNet[i].cout;
    return o;
}

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

struct Bufs {
    uint16_t *x0, *e1a, *cat1, *p1, *e2a, *cat2, *p2, *e3a, *e3b, *d2, *d1;
    float* r;
    uint16_t* wf[kLayers];
    uint16_t* wb[kLayers];
    // training
    uint16_t *g_r, *g_d1, *g_cat1, *g_d2, *g_cat2, *g_e3b, *g_e3a, *g_p2, *g_e2b, *g_e2a, *g_p1, *g_e1b, *g_e1a;
    float *part, *cnt_part, *loss_part, *n_hole;
    int chunks1, chunks2, chunks3;
    size_t bytes;
};

int chunk_rows(int rows) { return std::max(1, (rows + 127) / 128); }

Bufs layout(int B, int H, int W, bool train, char* base) {
    Layout L;
    Bufs f{};
    const size_t h1 = (size_t)H * W, h2 = h1 / 4, h3 = h1 / 16;
    auto bf = [&](size_t elems) { return (uint16_t*)(base + L.take(elems * 2)); };
    auto fl = [&](size_t elems) { return (float*)(base + L.take(elems * 4)); };
    f.x0 = bf(B * 8 * h1);
    f.e1a = bf(B * 16 * h1);
    f.cat1 = bf(B * 48 * h1);
    f.p1 = bf(B * 16 * h2);
    f.e2a = bf(B * 32 * h2);
    f.cat2 = bf(B * 96 * h2);
    f.p2 = bf(B * 32 * h3);
    f.e3a = bf(B * 64 * h3);
    f.e3b = bf(B * 64 * h3);
    f.d2 = bf(B * 32 * h2);
    f.d1 = bf(B * 16 * h1);
    f.r = fl(B * 4 * h1);
    for (int l = 0; l < kLayers; ++l) {
        f.wf[l] = bf((size_t)pad16(kNet[l].cout) * pad32(9 * pad16(kNet[l].cin)));
        f.wb[l] = bf((size_t)pad16(kNet[l].cin) * pad32(9 * pad16(kNet[l].cout)));
    }
    f.cnt_part = fl((B * h1 + 255) / 256);
    f.loss_part = fl((B * h1 + 255) / 256);
    f.n_hole = fl(1);
    if (train) {
        f.g_r = bf(B * 8 * h1);
        f.g_d1 = bf(B * 16 * h1);
        f.g_cat1 = bf(B * 48 * h1);
        f.g_d2 = bf(B * 32 * h2);
        f.g_cat2 = bf(B * 96 * h2);
        f.g_e3b = bf(B * 64 * h3);
        f.g_e3a = bf(B * 64 * h3);
        f.g_p2 = bf(B * 32 * h3);
        f.g_e2b = bf(B * 32 * h2);
        f.g_e2a = bf(B * 32 * h2);
        f.g_p1 = bf(B * 16 * h2);
        f.g_e1b = bf(B * 16 * h1);
        f.g_e1a = bf(B * 16 * h1);
        const int rows1 = B * H, rows2 = B * H / 2, rows3 = B * H / 4;
        f.chunks1 = (rows1 + chunk_rows(rows1) - 1) / chunk_rows(rows1);
        f.chunks2 = (rows2 + chunk_rows(rows2) - 1) / chunk_rows(rows2);
        f.chunks3 = (rows3 + chunk_rows(rows3) - 1) / chunk_rows(rows3);
        size_t mx = 0;
        const int lvl[kLayers] = {1, 1, 2, 2, 3, 3, 2, 1, 1};
        for (int l = 0; l < kLayers; ++l) {
            const int ch = lvl[l] == 1 ? f.chunks1 : lvl[l] == 2 ? f.chunks2 : f.chunks3;
            mx = std::max(mx, (size_t)ch * kNet[l].cout * (kNet[l].cin * 9 + 1));
        }
        f.part = fl(mx);
    }
    f.bytes = L.off;
    return f;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// The staged channel counts the convolution kernel is built for.
constexpr bool conv_cpad_ok(int cpad) { return cpad == 16 || cpad == 32 || cpad == 48 || cpad == 64 || cpad == 96; }
constexpr bool net_cpads_ok() {
    for (int l = 0; l < kLayers; ++l)
        if (!conv_cpad_ok(pad16(kNet[l].cin)) || !conv_cpad_ok(pad16(kNet[l].cout))) return false;
    return true;
}
static_assert(net_cpads_ok(), "every layer's input and output width needs a convolution instance");

template <int CPAD, int MT, int R>
void launch_conv(hipStream_t s, int B, const ConvArgs& a) {
    const int groups = (a.cout + 16 * MT - 1) / (16 * MT);
    hipLaunchKernelGGL((k_conv3x3<CPAD, MT, R>), dim3((a.W + 63) / 64, (a.H + R - 1) / R, B * groups), dim3(256),
                       conv_lds_bytes(CPAD, R), s, a);
}

// mt <= 2 for the tall shapes (more tiles would not fit in registers).
template <int CPAD>
constexpr bool tall_rows(int r) { return r == 8 || (CPAD > 64 && r == 4); }

template <int CPAD, int R>
void launch_conv(hipStream_t s, int B, int mt, const ConvArgs& a) {
    if constexpr (tall_rows<CPAD>(R)) {
        if (mt == 1)
            launch_conv<CPAD, 1, R>(s, B, a);
        else
            launch_conv<CPAD, 2, R>(s, B, a);
    } else {
        switch (mt) {
            case 1: launch_conv<CPAD, 1, R>(s, B, a); break;
            case 2: launch_conv<CPAD, 2, R>(s, B, a); break;
            case 3: launch_conv<CPAD, 3, R>(s, B, a); break;
            default: launch_conv<CPAD, 4, R>(s, B, a); break;
        }
    }
}

// Block shape: four output rows per block where that still leaves at least
// six blocks per CU (they share the two halo rows and each weight operand),
// else two; then fewer output tiles per block until there are at least two
// blocks per CU, since the coarse levels have few pixels (at 200x150, two
// tiles over 600 blocks beat one tile over 1200: 11.6 against 16.7 us for
// the 64-channel layer).  bgs_repair_set_block_shape may fix either choice
// (0: automatic), and may ask for eight rows (inputs of up to 64 channels)
// or four rows of 96 channels, which take at most two output tiles.
std::atomic<int> g_rows{0}, g_tiles{0};

template <int CPAD>
void launch_conv(hipStream_t s, int B, const ConvArgs& a) {
    const int tiles = (a.cout + 15) / 16;
    auto nblk = [&](int r, int mt) {
        return (int64_t)((a.W + 63) / 64) * ((a.H + r - 1) / r) * B * ((tiles + mt - 1) / mt);
    };
    const int fr = g_rows.load(), ft = g_tiles.load();
    int mt = std::min(4, tiles);
    // Largest row count offered for this width (a workgroup may take up to
    // 160 KB of LDS): 8 rows up to 64 staged channels (95 KB at 64), 4 rows
    // of 96 (85 KB).
    constexpr int kMaxRows = CPAD <= 64 ? 8 : 4;
    // Automatic: 96 staged channels keep two rows (four take 85 KB of LDS,
    // one block per CU, and measured slower: 211 against 194 us at
    // 1032x1104); taller blocks than four rows measured no better.
    int r = std::min(kMaxRows, fr ? fr : (CPAD <= 64 && nblk(4, mt) >= 6 * 256) ? 4 : 2);
    if (ft)
        mt = std::min(ft, tiles);
    else
        while (mt > 1 && nblk(r, mt) < 2 * 256) mt = (mt + 1) / 2;
    if (mt > 2 && tall_rows<CPAD>(r)) r = r == 8 && CPAD <= 64 ? 4 : 2;
    if (r == 8)
        launch_conv<CPAD, (kMaxRows >= 8 ? 8 : 2)>(s, B, mt, a);
    else if (r == 4)
        launch_conv<CPAD, (kMaxRows >= 4 ? 4 : 2)>(s, B, mt, a);
    else
        launch_conv<CPAD, 2>(s, B, mt, a);
}

// A bf16 activation or gradient tensor [B][H][W] of pixels holding ps
// elements (bs per image), from channel 0 of a slice.
struct View {
    uint16_t* p;
    int64_t bs;
    int ps;
    View at(int channel) const { return View{p + channel, bs, ps}; }
};
const View kNone{nullptr, 0, 0};

// up (optional, with up_c): the half-resolution source of the first up_c
// input channels, read through the nearest 2x upsample.  out_f (fp32
// planes) replaces out when set.
void conv(hipStream_t s, int B, int H, int W, int l, bool transpose, const Bufs& f, View in, const float* params,
          View out, float* out_f, View mask, View up = kNone, int up_c = 0, View pool = kNone) {
    ConvArgs a{};
    a.in = in.p;
    a.in_bs = in.bs;
    a.in_ps = in.ps;
    a.cin = transpose ? kNet[l].cout : kNet[l].cin;
    a.up = up.p;
    a.up_bs = up.bs;
    a.up_ps = up.ps;
    a.up_c = up.p ? up_c : 0;
    a.cout = transpose ? kNet[l].cin : kNet[l].cout;
    a.w = transpose ? f.wb[l] : f.wf[l];
    const int cpad = pad16(a.cin);
    a.kpad = pad32(9 * cpad);
    a.bias = transpose ? nullptr : params + param_offset(l) + (int64_t)kNet[l].cout * kNet[l].cin * 9;
    a.out = out.p;
    a.out_bs = out_f ? (int64_t)a.cout * H * W : out.bs;
    a.out_ps = out.ps;
    a.out_f = out_f;
    a.mask = mask.p;
    a.mask_bs = mask.bs;
    a.mask_ps = mask.ps;
    a.pool = pool.p;
    a.pool_bs = pool.bs;
    a.pool_ps = pool.ps;
    a.relu = transpose ? 0 : kNet[l].relu;
    a.H = H;
    a.W = W;
    switch (cpad) {
        case 16: launch_conv<16>(s, B, a); break;
        case 32: launch_conv<32>(s, B, a); break;
        case 48: launch_conv<48>(s, B, a); break;
        case 64: launch_conv<64>(s, B, a); break;
        default: launch_conv<96>(s, B, a); break;  // the only other width (static_assert above)
    }
}

void wgrad(hipStream_t s, int B, int H, int W, int l, const Bufs& f, View g, View in, int chunks, float* grad) {
    WgradArgs a{};
    a.g = g.p;
    a.g_bs = g.bs;
    a.g_ps = g.ps;
    a.cout = kNet[l].cout;
    a.in = in.p;
    a.in_bs = in.bs;
    a.in_ps = in.ps;
    a.cin = kNet[l].cin;
    a.B = B;
    a.H = H;
    a.W = W;
    a.rows = chunk_rows(B * H);
    a.part = f.part;
    const int K = a.cin * 9;
    const int nt = (K + 1 + 15) / 16;
    hipLaunchKernelGGL(k_wgrad, dim3((nt + 3) / 4, chunks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)(((int64_t)a.cout * (K + 1) + 63) / 64)), dim3(256), 0, s,
                       (const float*)f.part, chunks, a.cout, K, grad + param_offset(l));
}

// The tensors of one pass, as views.
struct Net {
    View x0, e1a, cat1, e1b, p1, e2a, cat2, e2b, p2, e3a, e3b, d2, d1;
    View g_r, g_d1, g_cat1, g_d2, g_cat2, g_e3b, g_e3a, g_p2, g_e2b, g_e2a, g_p1, g_e1b, g_e1a;
};

// Training keeps each decoder's concatenated input whole (the weight
// gradient reads it), the skip connection in its last channels; inference
// stores the skip tensors dense, in the same memory.
Net views(const Bufs& f, int H, int W, bool train) {
    const int64_t h1 = (int64_t)H * W, h2 = h1 / 4, h3 = h1 / 16;
    auto v = [](uint16_t* p, int c, int64_t hw) { return View{p, c * hw, c}; };
    Net n;
    n.x0 = v(f.x0, 8, h1);
    n.e1a = v(f.e1a, 16, h1);
    n.cat1 = v(f.cat1, 48, h1);  // up(d2) in channels 0-31, e1b in 32-47
    n.e1b = train ? n.cat1.at(32) : v(f.cat1, 16, h1);
    n.p1 = v(f.p1, 16, h2);
    n.e2a = v(f.e2a, 32, h2);
    n.cat2 = v(f.cat2, 96, h2);  // up(e3b) in channels 0-63, e2b in 64-95
    n.e2b = train ? n.cat2.at(64) : v(f.cat2, 32, h2);
    n.p2 = v(f.p2, 32, h3);
    n.e3a = v(f.e3a, 64, h3);
    n.e3b = v(f.e3b, 64, h3);
    n.d2 = v(f.d2, 32, h2);
    n.d1 = v(f.d1, 16, h1);
    n.g_r = v(f.g_r, 8, h1);
    n.g_d1 = v(f.g_d1, 16, h1);
    n.g_cat1 = v(f.g_cat1, 48, h1);
    n.g_d2 = v(f.g_d2, 32, h2);
    n.g_cat2 = v(f.g_cat2, 96, h2);
    n.g_e3b = v(f.g_e3b, 64, h3);
    n.g_e3a = v(f.g_e3a, 64, h3);
    n.g_p2 = v(f.g_p2, 32, h3);
    n.g_e2b = v(f.g_e2b, 32, h2);
    n.g_e2a = v(f.g_e2a, 32, h2);
    n.g_p1 = v(f.g_p1, 16, h2);
    n.g_e1b = v(f.g_e1b, 16, h1);
    n.g_e1a = v(f.g_e1a, 16, h1);
    return n;
}

inline unsigned chan_blocks(int B, int64_t pixels, int C) { return blocks((int64_t)B * pixels * (C / 8)); }

void forward(hipStream_t s, int B, int H, int W, const float* params, const float* rgb, const float* z,
             const uint8_t* hole, const Bufs& f, bool train) {
    // Forward weights always; the transposed ones only for the input
    // gradient of training.
    PackJobs J{};
    J.start[0] = 0;
    for (int t = 0; t < (train ? 2 : 1); ++t)
        for (int l = 0; l < kLayers; ++l) {
            const int ci = kNet[l].cin, co = kNet[l].cout;
            PackJob& P = J.job[J.n];
            P.w = params + param_offset(l);
            P.out = t ? f.wb[l] : f.wf[l];
            P.cin = ci;
            P.cout = co;
            P.transpose = t;
            P.cpad = pad16(t ? co : ci);
            P.kpad = pad32(9 * P.cpad);
            J.start[J.n + 1] = J.start[J.n] + pad16(t ? ci : co) * P.kpad;
            ++J.n;
        }
    hipLaunchKernelGGL(k_pack, dim3(blocks(J.start[J.n])), dim3(256), 0, s, J);
    const Net n = views(f, H, W, train);
    const int64_t h1 = (int64_t)H * W, h2 = h1 / 4;
    const int H2 = H / 2, W2 = W / 2, H3 = H / 4, W3 = W / 4;
    hipLaunchKernelGGL(k_input, dim3(blocks(B * h1)), dim3(256), 0, s, rgb, z, hole, B, (int)h1, f.x0);
    conv(s, B, H, W, E1A, false, f, n.x0, params, n.e1a, nullptr, kNone);
    // The encoders' second convolutions also store the pooled output.
    conv(s, B, H, W, E1B, false, f, n.e1a, params, n.e1b, nullptr, kNone, kNone, 0, n.p1);
    conv(s, B, H2, W2, E2A, false, f, n.p1, params, n.e2a, nullptr, kNone);
    conv(s, B, H2, W2, E2B, false, f, n.e2a, params, n.e2b, nullptr, kNone, kNone, 0, n.p2);
    conv(s, B, H3, W3, E3A, false, f, n.p2, params, n.e3a, nullptr, kNone);
    conv(s, B, H3, W3, E3B, false, f, n.e3a, params, n.e3b, nullptr, kNone);
    // The decoders read their upsampled channels straight from the coarser
    // level; training also stores the upsample, which the weight gradient
    // reads.
    if (train)
        hipLaunchKernelGGL(k_up, dim3(chan_blocks(B, h2, 64)), dim3(256), 0, s, f.e3b, B, 64, H3, W3, n.cat2.p,
                           n.cat2.bs, n.cat2.ps);
    conv(s, B, H2, W2, D2, false, f, n.e2b, params, n.d2, nullptr, kNone, n.e3b, 64);
    if (train)
        hipLaunchKernelGGL(k_up, dim3(chan_blocks(B, h1, 32)), dim3(256), 0, s, f.d2, B, 32, H2, W2, n.cat1.p,
                           n.cat1.bs, n.cat1.ps);
    conv(s, B, H, W, D1, false, f, n.e1b, params, n.d1, nullptr, kNone, n.d2, 32);
    conv(s, B, H, W, OUT, false, f, n.d1, params, kNone, f.r, kNone);
}

void backward(hipStream_t s, int B, int H, int W, const float* params, const Bufs& f, float* grad) {
    const Net n = views(f, H, W, true);
    const int64_t h1 = (int64_t)H * W, h2 = h1 / 4;
    const int H2 = H / 2, W2 = W / 2, H3 = H / 4, W3 = W / 4;
    wgrad(s, B, H, W, OUT, f, n.g_r, n.d1, f.chunks1, grad);
    conv(s, B, H, W, OUT, true, f, n.g_r, params, n.g_d1, nullptr, n.d1);
    wgrad(s, B, H, W, D1, f, n.g_d1, n.cat1, f.chunks1, grad);
    conv(s, B, H, W, D1, true, f, n.g_d1, params, n.g_cat1, nullptr, kNone);
    hipLaunchKernelGGL(k_up_grad, dim3(chan_blocks(B, h2, 32)), dim3(256), 0, s, n.g_cat1.p, n.g_cat1.bs, n.g_cat1.ps,
                       B, 32, H, W, f.d2, f.g_d2);
    wgrad(s, B, H2, W2, D2, f, n.g_d2, n.cat2, f.chunks2, grad);
    conv(s, B, H2, W2, D2, true, f, n.g_d2, params, n.g_cat2, nullptr, kNone);
    hipLaunchKernelGGL(k_up_grad, dim3(chan_blocks(B, h2 / 4, 64)), dim3(256), 0, s, n.g_cat2.p, n.g_cat2.bs,
                       n.g_cat2.ps, B, 64, H2, W2, f.e3b, f.g_e3b);
    wgrad(s, B, H3, W3, E3B, f, n.g_e3b, n.e3a, f.chunks3, grad);
    conv(s, B, H3, W3, E3B, true, f, n.g_e3b, params, n.g_e3a, nullptr, n.e3a);
    wgrad(s, B, H3, W3, E3A, f, n.g_e3a, n.p2, f.chunks3, grad);
    conv(s, B, H3, W3, E3A, true, f, n.g_e3a, params, n.g_p2, nullptr, kNone);
    const View sk2 = n.g_cat2.at(64), sk1 = n.g_cat1.at(32);
    hipLaunchKernelGGL(k_merge, dim3(chan_blocks(B, h2, 32)), dim3(256), 0, s, sk2.p, sk2.bs, sk2.ps, f.g_p2, n.e2b.p,
                       n.e2b.bs, n.e2b.ps, B, 32, H2, W2, f.g_e2b);
    wgrad(s, B, H2, W2, E2B, f, n.g_e2b, n.e2a, f.chunks2, grad);
    conv(s, B, H2, W2, E2B, true, f, n.g_e2b, params, n.g_e2a, nullptr, n.e2a);
    wgrad(s, B, H2, W2, E2A, f, n.g_e2a, n.p1, f.chunks2, grad);
    conv(s, B, H2, W2, E2A, true, f, n.g_e2a, params, n.g_p1, nullptr, kNone);
    hipLaunchKernelGGL(k_merge, dim3(chan_blocks(B, h1, 16)), dim3(256), 0, s, sk1.p, sk1.bs, sk1.ps, f.g_p1, n.e1b.p,
                       n.e1b.bs, n.e1b.ps, B, 16, H, W, f.g_e1b);
    wgrad(s, B, H, W, E1B, f, n.g_e1b, n.e1a, f.chunks1, grad);
    conv(s, B, H, W, E1B, true, f, n.g_e1b, params, n.g_e1a, nullptr, n.e1a);
    wgrad(s, B, H, W, E1A, f, n.g_e1a, n.x0, f.chunks1, grad);
}

bool sizes_ok(int B, int H, int W) { return B >= 1 && B <= 1000 && H >= 4 && W >= 4 && H % 4 == 0 && W % 4 == 0 && H <= 8192 && W <= 8192; }

int32_t launched() { return hipGetLastError() == hipSuccess ? BGS_OK : BGS_ERR_HIP; }

}  // namespace

extern "C" {

BGS_API int32_t bgs_repair_num_params(int64_t* n) {
    if (!n) return BGS_ERR_INVALID_ARG;
    *n = param_offset(kLayers);
    return BGS_OK;
}

BGS_API int32_t bgs_repair_workspace_size(int32_t batch, int32_t height, int32_t width, int32_t train, size_t* bytes) {
    if (!bytes || !sizes_ok(batch, height, width) || (train != 0 && train != 1)) return BGS_ERR_INVALID_ARG;
    *bytes = layout(batch, height, width, train != 0, nullptr).bytes;
    return BGS_OK;
}

BGS_API int32_t bgs_repair_forward(const float* params, int32_t batch, int32_t height, int32_t width,
                                   const float* rgb, const float* z, const uint8_t* hole, float* rgb_out,
                                   float* err_out, void* ws, size_t ws_bytes, void* hip_stream) {
    if (!params || !rgb || !z || !hole || !rgb_out || !ws || !sizes_ok(batch, height, width))
        return BGS_ERR_INVALID_ARG;
    const Bufs f = layout(batch, height, width, false, (char*)ws);
    if (ws_bytes < f.bytes) return BGS_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)hip_stream;
    (void)hipGetLastError();
    forward(s, batch, height, width, params, rgb, z, hole, f, false);
    const int64_t np = (int64_t)batch * height * width;
    hipLaunchKernelGGL(k_output, dim3(blocks(np)), dim3(256), 0, s, rgb, hole, (const float*)f.r, batch,
                       height * width, rgb_out, err_out);
    return launched();
}

BGS_API int32_t bgs_repair_hole_error(const float* err, const uint8_t* hole, int32_t batch, int32_t height,
                                      int32_t width, float* out, float* scratch, void* hip_stream) {
    static_assert(kErrParts == 256, "one part per thread of the second step");
    if (!err || !hole || !out || !scratch || batch < 1 || batch > 1000 || height < 1 || width < 1 || height > 16384 ||
        width > 16384)
        return BGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_err_part, dim3(kErrParts, batch), dim3(256), 0, s, err, hole, (int64_t)height * width,
                       scratch);
    hipLaunchKernelGGL(k_err_mean, dim3(batch), dim3(256), 0, s, (const float*)scratch, out);
    return launched();
}

BGS_API int32_t bgs_repair_grad(const float* params, int32_t batch, int32_t height, int32_t width, const float* rgb,
                                const float* z, const uint8_t* hole, const float* target, float* grad, float* loss,
                                float* rgb_out, void* ws, size_t ws_bytes, void* hip_stream) {
    if (!params || !rgb || !z || !hole || !target || !grad || !loss || !ws || !sizes_ok(batch, height, width))
        return BGS_ERR_INVALID_ARG;
    const Bufs f = layout(batch, height, width, true, (char*)ws);
    if (ws_bytes < f.bytes) return BGS_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)hip_stream;
    (void)hipGetLastError();
    forward(s, batch, height, width, params, rgb, z, hole, f, true);
    const int HW = height * width;
    const int64_t np = (int64_t)batch * HW;
    hipLaunchKernelGGL(k_count, dim3(blocks(np)), dim3(256), 0, s, hole, np, f.cnt_part);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, (const float*)f.cnt_part, (int)blocks(np), (const float*)nullptr,
                       f.n_hole);
    hipLaunchKernelGGL(k_loss, dim3(blocks(np)), dim3(256), 0, s, rgb, hole, (const float*)f.r, target,
                       (const float*)f.n_hole, batch, HW, rgb_out, f.g_r, f.loss_part);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, (const float*)f.loss_part, (int)blocks(np),
                       (const float*)f.n_hole, loss);
    backward(s, batch, height, width, params, f, grad);
    return launched();
}

BGS_API int32_t bgs_repair_set_block_shape(int32_t rows, int32_t tiles) {
    if (!(rows == 0 || rows == 2 || rows == 4 || rows == 8) || tiles < 0 || tiles > 4) return BGS_ERR_INVALID_ARG;
    g_rows.store(rows);
    g_tiles.store(tiles);
    return BGS_OK;
}

BGS_API int32_t bgs_repair_adam(float* params, const float* grad, float* m, float* v, int64_t n, int32_t step,
                                float lr, float beta1, float beta2, float eps, void* hip_stream) {
    if (!params || !grad || !m || !v || n < 1 || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return BGS_ERR_INVALID_ARG;
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(256), 0, (hipStream_t)hip_stream, params, grad, m, v, n, lr,
                       beta1, beta2, eps, c1, c2);
    return launched();
}

}  // extern "C"
