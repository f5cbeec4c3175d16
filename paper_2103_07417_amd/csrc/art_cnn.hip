// art_cnn.hip -- learned refinement proposal: a 4-layer 3x3 convolutional
// network (channels 3 -> 32 -> 32 -> 32 -> 15) run and trained with BF16 MFMA
// (gfx950's v_mfma_f32_32x32x16_bf16: 32 x 32 outputs, depth 16 per
// instruction) and FP32 accumulation.
//
// The network sees the level-l vertex grid of an adaptive render (log
// intensity, minimum radius, equatorial crossings) and predicts, for every
// level-l vertex, whether the 3 points it owns at level l+1 and the 12 at
// level l+2 will be ray traced.  The refinement criterion of Sec. 3.2
// (Eqs. 5-6) stays the judge and the fallback.
//
// Layouts.  Activations are NHWC in BF16 with the channel count padded to a
// multiple of 8 (input 3 -> 8, hidden 32, output gradient 15 -> 16), so a
// lane's 8 consecutive reduction elements are one 16-byte load.  The GEMM
// depth is ordered tap-major, k = (dy * 3 + dx) * C_pad + c, and cut into
// 8-channel chunks; one 16-deep MFMA step takes two consecutive chunks, one
// per half-wave (for 8 channels: two taps; a ninth tap is paired with zeros).  Logits are FP32 NCHW
// ([b][15][H][W]) like labels.  Master weights stay FP32 in the order
// W[c_out][c_in][3][3] and are packed into BF16 GEMM matrices after each
// update.
//
// Convolution = implicit GEMM D[position][c_out] = sum_k A[position][k]
// B[k][c_out]: one wave per 32 positions of one row x 32 output channels.
// Weight gradients are the GEMM dW[c_out][k] = sum_position dZ A, reduced
// over position chunks in a fixed order (deterministic).  Input gradients are
// the forward convolution of dZ with the flipped, transposed weights.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "art_cnn.hpp"

namespace art {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// D += A B on a 32 x 32 tile, depth 16: lane l supplies A[l % 32][8 (l / 32)
// .. + 7] and B[8 (l / 32) .. + 7][l % 32]; D[8 (j / 4) + 4 (l / 32) + j % 4]
// [l % 32] is element j of its accumulator.
__device__ __forceinline__ floatx16 mfma16(shortx8 a, shortx8 b, floatx16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   c, 0, 0, 0);
}
__device__ __forceinline__ shortx8 join8(bf16x4 lo, bf16x4 hi)
{
    return shortx8{ lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3] };
}

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);          // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ------------------------------------------------------------------ forward
// in [B][H][W][cin_pad] bf16; Wm [32][Kp] bf16 (row = output channel, k
// tap-major); bias [co].  Output by mode (see art_cnn.hpp); bf16 outputs are
// NHWC with 32 channels, FP32 logits NCHW with co channels.
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ in, int cin_pad, int B, int H,
                                                  int W, const uint16_t* __restrict__ Wm, int Kp,
                                                  const float* __restrict__ bias, int co, int mode,
                                                  void* __restrict__ out, const uint16_t* __restrict__ mask)
{
    const int lane = threadIdx.x & 63;
    const long long wave = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tiles_x = (W + 31) >> 5;
    const long long row = wave / tiles_x;                 // b * H + y
    if (row >= (long long)B * H) return;                  // uniform per wave
    const int b = (int)(row / H), y = (int)(row - (long long)b * H);
    const int x0 = (int)(wave - row * tiles_x) << 5;
    const int m = lane & 31, kb = lane >> 5;
    const int x = x0 + m;
    const long long HW = (long long)H * W;
    const uint16_t* inb = in + (long long)b * HW * cin_pad;
    floatx16 acc;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
    // depth in 8-channel chunks, two per 16-deep step (one per half-wave);
    // the next step's operands are loaded before this step's MFMA
    const int nch = (9 * cin_pad) >> 3;
    const int nst = (nch + 1) >> 1;
    auto load = [&](int st, shortx8& a, shortx8& bw) {
        const int ch = 2 * st + kb;
        a = shortx8{ 0, 0, 0, 0, 0, 0, 0, 0 };
        bw = a;
        if (ch < nch) {
            const int k0 = ch << 3, tap = k0 / cin_pad, c8 = k0 - tap * cin_pad;
            const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
            if (x < W && yy >= 0 && yy < H && xx >= 0 && xx < W)
                a = *(const shortx8*)(inb + ((long long)yy * W + xx) * cin_pad + c8);
            bw = *(const shortx8*)(Wm + (long long)m * Kp + k0);
        }
    };
    shortx8 A[2], Bw[2];
    load(0, A[0], Bw[0]);
    for (int st = 0; st < nst; ++st) {
        if (st + 1 < nst) load(st + 1, A[(st + 1) & 1], Bw[(st + 1) & 1]);
        acc = mfma16(A[st & 1], Bw[st & 1], acc);
    }
    // D[row][col]: col = lane % 32 (output channel), row = 8 (j/4) + 4 (lane/32) + j%4
    const int oc = m;
    if (mode == 1 && oc >= co) return;
    const float bb = (mode == 2 || oc >= co) ? 0.0f : bias[oc];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int xo = x0 + 8 * (j >> 2) + 4 * kb + (j & 3);
        if (xo >= W) continue;
        const long long pos = (long long)y * W + xo;
        const float v = acc[j] + bb;
        if (mode == 0) {
            ((uint16_t*)out)[((long long)b * HW + pos) * 32 + oc] = f2bf(v > 0.0f ? v : 0.0f);
        } else if (mode == 1) {
            ((float*)out)[((long long)b * co + oc) * HW + pos] = v;
        } else {
            const long long o = ((long long)b * HW + pos) * 32 + oc;
            ((uint16_t*)out)[o] = f2bf(bf2f(mask[o]) > 0.0f ? v : 0.0f);
        }
    }
}

// The same convolution with its operands staged in LDS (CIN = 8 or 32).  A
// block of four waves copies the weight matrix once ([32][9 CIN], rows padded
// by 4) and then walks kConvTiles rounds of four consecutive 32-position
// tiles, one per wave: each wave stages its tile's 3 x 34 input halo (rows
// y-1..y+1, zero outside the image, positions padded by 4 channels) and runs
// the nine taps from LDS.  The next round's halo is loaded into registers
// before this round's MFMAs, so its global reads overlap them; reusing the
// staged weights over the rounds removes the per-tile weight copy that
// bounded a one-tile block.  Halo lanes of a tile beyond the image width
// produce output rows that are discarded.
constexpr int kConvTiles = 8;

template <int CIN>
__global__ __launch_bounds__(256) void k_conv_fwd_lds(const uint16_t* __restrict__ in, int B, int H, int W,
                                                      const uint16_t* __restrict__ Wm,
                                                      const float* __restrict__ bias, int co, int mode,
                                                      void* __restrict__ out, const uint16_t* __restrict__ mask)
{
    constexpr int KP = 9 * CIN;          // GEMM depth
    constexpr int WS = KP + 4;           // staged weight row stride (bf16)
    constexpr int CS = CIN + 4;          // staged position stride (bf16)
    constexpr int NPOS = 3 * 34;
    constexpr int NA = NPOS * (CIN / 4); // 8-byte chunks of a wave's halo
    constexpr int NAL = (NA + 63) / 64;  // per lane
    constexpr int NW = 32 * (KP / 4);    // 8-byte chunks of the weights
    constexpr int NWT = (NW + 255) / 256;
    constexpr int NCH = KP / 8;          // 8-channel chunks of the depth
    __shared__ __align__(16) uint16_t sW[32 * WS];
    __shared__ __align__(16) uint16_t sA[4][NPOS * CS];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int tiles_x = (W + 31) >> 5;
    const long long ntiles = (long long)B * H * tiles_x;
    const long long HW = (long long)H * W;
    const int m = lane & 31, kb = lane >> 5;
    const int oc = m;
    const float bb = (mode == 2 || oc >= co) ? 0.0f : bias[oc < co ? oc : 0];
    uint16_t* a_s = sA[wv];

    // tile of round r: (image b, row y, first column x0), or invalid
    auto tile_of = [&](int r, int& b, int& y, int& x0) {
        const long long t = ((long long)blockIdx.x * kConvTiles + r) * 4 + wv;
        if (t >= ntiles) return false;
        const long long row = t / tiles_x;
        b = (int)(row / H);
        y = (int)(row - (long long)b * H);
        x0 = (int)(t - row * tiles_x) << 5;
        return true;
    };
    bf16x4 av_[NAL];
    auto load_halo = [&](int r) {
        int b, y, x0;
        const bool ok = tile_of(r, b, y, x0);
        const uint16_t* inb = in + (long long)(ok ? b : 0) * HW * CIN;
#pragma unroll
        for (int t = 0; t < NAL; ++t) {
            const int q = lane + 64 * t;
            av_[t] = bf16x4{ 0, 0, 0, 0 };
            if (ok && q < NA) {
                const int pos = q / (CIN / 4), c4 = q - pos * (CIN / 4);
                const int pr = pos / 34, pc = pos - pr * 34;
                const int yy = y - 1 + pr, xx = x0 - 1 + pc;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    av_[t] = *(const bf16x4*)(inb + ((long long)yy * W + xx) * CIN + 4 * c4);
            }
        }
    };
    {
        bf16x4 wv_[NWT];
#pragma unroll
        for (int t = 0; t < NWT; ++t) {
            const int q = threadIdx.x + 256 * t;
            wv_[t] = bf16x4{ 0, 0, 0, 0 };
            if (q < NW) {
                const int r = q / (KP / 4), c4 = q - r * (KP / 4);
                wv_[t] = *(const bf16x4*)(Wm + (long long)r * KP + 4 * c4);
            }
        }
        load_halo(0);
#pragma unroll
        for (int t = 0; t < NWT; ++t) {
            const int q = threadIdx.x + 256 * t;
            if (q < NW) {
                const int r = q / (KP / 4), c4 = q - r * (KP / 4);
                *(bf16x4*)&sW[r * WS + 4 * c4] = wv_[t];
            }
        }
    }
    for (int r = 0; r < kConvTiles; ++r) {
        if (r > 0) __syncthreads();           // every wave is done reading its halo slot
#pragma unroll
        for (int t = 0; t < NAL; ++t) {
            const int q = lane + 64 * t;
            if (q < NA) {
                const int pos = q / (CIN / 4), c4 = q - pos * (CIN / 4);
                *(bf16x4*)&a_s[pos * CS + 4 * c4] = av_[t];
            }
        }
        __syncthreads();                      // halos (and, in the first tile round, weights) staged
        int b, y, x0;
        const bool ok = tile_of(r, b, y, x0);
        if (r + 1 < kConvTiles) load_halo(r + 1);
        if (ok) {
            floatx16 acc;
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
            // two 8-channel chunks per 16-deep step: this half-wave takes
            // chunk 2 st + kb (a chunk past the depth is zero)
#pragma unroll
            for (int st = 0; st < (NCH + 1) / 2; ++st) {
                const int ch = 2 * st + kb;
                const int tap = (8 * ch) / CIN, c8 = 8 * ch - tap * CIN;
                const int dy = tap / 3, dx = tap - 3 * dy;
                shortx8 a = shortx8{ 0, 0, 0, 0, 0, 0, 0, 0 }, bw = a;
                if (ch < NCH) {
                    const uint16_t* pa = &a_s[(dy * 34 + m + dx) * CS + c8];
                    const uint16_t* pb = &sW[m * WS + 8 * ch];
                    a = join8(*(const bf16x4*)pa, *(const bf16x4*)(pa + 4));
                    bw = join8(*(const bf16x4*)pb, *(const bf16x4*)(pb + 4));
                }
                acc = mfma16(a, bw, acc);
            }
            if (!(mode == 1 && oc >= co)) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int xo = x0 + 8 * (j >> 2) + 4 * kb + (j & 3);
                    if (xo >= W) continue;
                    const long long pos = (long long)y * W + xo;
                    const float v = acc[j] + bb;
                    if (mode == 0) {
                        ((uint16_t*)out)[((long long)b * HW + pos) * 32 + oc] = f2bf(v > 0.0f ? v : 0.0f);
                    } else if (mode == 1) {
                        ((float*)out)[((long long)b * co + oc) * HW + pos] = v;
                    } else {
                        const long long o = ((long long)b * HW + pos) * 32 + oc;
                        ((uint16_t*)out)[o] = f2bf(bf2f(mask[o]) > 0.0f ? v : 0.0f);
                    }
                }
            }
        }
    }
}

hipError_t cnn_conv_fwd(const uint16_t* in, int cin_pad, int B, int H, int W, const uint16_t* Wm, int Kp,
                        const float* bias, int co, int mode, void* out, const uint16_t* mask,
                        hipStream_t s)
{
    // the kernels read the depth in 8-channel chunks of at most 32 channels
    if (cin_pad < 8 || cin_pad > 32 || (cin_pad & 7) || Kp != 9 * cin_pad || co < 1 || co > 32)
        return hipErrorInvalidValue;
    const long long waves = (long long)B * H * ((W + 31) / 32);
    const long long blocks = (waves + 3) / 4;
    const long long lds_blocks = (waves + 4 * kConvTiles - 1) / (4 * kConvTiles);
    if (cin_pad == 32)
        hipLaunchKernelGGL(k_conv_fwd_lds<32>, dim3((unsigned)lds_blocks), dim3(256), 0, s, in, B, H, W, Wm, bias,
                           co, mode, out, mask);
    else if (cin_pad == 8)
        hipLaunchKernelGGL(k_conv_fwd_lds<8>, dim3((unsigned)lds_blocks), dim3(256), 0, s, in, B, H, W, Wm, bias,
                           co, mode, out, mask);
    else
        hipLaunchKernelGGL(k_conv_fwd, dim3((unsigned)blocks), dim3(256), 0, s, in, cin_pad, B, H, W, Wm, Kp,
                           bias, co, mode, out, mask);
    return hipGetLastError();
}

// ------------------------------------------------------- weight gradients
// Positions are split into nchunks chunks of clen (a multiple of 16); one wave
// per (chunk, 32-wide tile of the tap-major depth k = tap * cin_pad + c)
// writes part[chunk][ktile][32 c_out][32 k].  A operand = dZ (rows = output
// channel), B operand = im2col(in) (columns = k, 32 consecutive channels of
// one shifted position per lane group); reduction over positions, whose
// (image, row, column) is advanced incrementally (no divisions in the loop).
__global__ __launch_bounds__(256) void k_conv_dw(const uint16_t* __restrict__ in, int ci, int cin_pad, int B,
                                                 int H, int W, const uint16_t* __restrict__ dZ, int co,
                                                 int cout_pad, float* __restrict__ part, float* __restrict__ dbpart,
                                                 int nchunks, long long clen)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int Kp = 9 * cin_pad;
    const int ktiles = (Kp + 31) >> 5;
    const int chunk = wave / ktiles;
    if (chunk >= nchunks) return;
    const int kt = wave - chunk * ktiles;
    const int m = lane & 31, kb = lane >> 5;
    const long long HW = (long long)H * W;
    const long long P = (long long)B * HW;
    const long long p0 = (long long)chunk * clen;
    const long long p1 = p0 + clen < P ? p0 + clen : P;
    floatx16 acc;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
    const int k = kt * 32 + m;                       // this lane's B column (tap-major)
    const int tap = k / cin_pad, c = k - tap * cin_pad;
    const bool kval = tap < 9 && c < ci;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    // (image, row, column) of the first position of each 16-position step
    int pb = (int)(p0 / HW);
    const long long q0 = p0 - (long long)pb * HW;
    int py = (int)(q0 / W), px = (int)(q0 - (long long)py * W);
    float sdb = 0.0f;                                // bias gradient partial (k tile 0 only)
    for (long long ps = p0; ps < p1; ps += 16) {
        shortx8 a, bv;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int o = 8 * kb + t;
            const long long p = ps + o;
            short av = 0, bw = 0;
            if (p < p1) {
                if (m < co) {
                    av = (short)dZ[p * cout_pad + m];
                    sdb += bf2f((uint16_t)av);
                }
                if (kval) {
                    int x = px + o, y = py, b = pb;
                    while (x >= W) { x -= W; ++y; }
                    while (y >= H) { y -= H; ++b; }
                    const int yy = y + dy, xx = x + dx;
                    if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                        bw = (short)in[((long long)b * HW + (long long)yy * W + xx) * cin_pad + c];
                }
            }
            a[t] = av;
            bv[t] = bw;
        }
        acc = mfma16(a, bv, acc);
        px += 16;
        while (px >= W) { px -= W; ++py; }
        while (py >= H) { py -= H; ++pb; }
    }
    float* Pp = part + ((long long)chunk * ktiles + kt) * 1024;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int row = 8 * (j >> 2) + 4 * kb + (j & 3);      // output channel
        Pp[row * 32 + m] = acc[j];
    }
    if (kt == 0) {
        // lanes m and m + 32 hold the two halves of channel m's positions
        const float other = __shfl_down(sdb, 32);
        if (kb == 0) dbpart[(long long)chunk * 32 + m] = sdb + other;
    }
}

// Deterministic two-stage sum over the position chunks.  Stage 1: thread
// (output e, slice sl) sums chunks sl, sl + S, sl + 2S, ... in order into
// red[sl][e]; outputs e < co * K are the weights in master order
// (e = o * K + c * 9 + tap, read from the tap-major partials), then co
// biases.  Stage 2 sums the S slices in order.
constexpr int kDwSlices = 16;

__global__ __launch_bounds__(256) void k_dw_reduce1(const float* __restrict__ part, const float* __restrict__ dbpart,
                                                    int nchunks, int ktiles, int co, int ci, int cin_pad,
                                                    float* __restrict__ red)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = blockIdx.y;
    const int K = ci * 9;
    const int nout = co * K + co;
    if (e >= nout) return;
    float s = 0.0f;
    if (e < co * K) {
        const int o = e / K, km = e - o * K;
        const int c = km / 9, tap = km - 9 * c;
        const int kp = tap * cin_pad + c;
        const int kt = kp >> 5, kk = kp & 31;
        for (int ch = sl; ch < nchunks; ch += kDwSlices)
            s += part[((long long)ch * ktiles + kt) * 1024 + o * 32 + kk];
    } else {
        const int o = e - co * K;
        for (int ch = sl; ch < nchunks; ch += kDwSlices) s += dbpart[(long long)ch * 32 + o];
    }
    red[(long long)sl * nout + e] = s;
}

__global__ __launch_bounds__(256) void k_dw_reduce2(const float* __restrict__ red, int co, int ci,
                                                    float* __restrict__ dW, float* __restrict__ db)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int K = ci * 9;
    const int nout = co * K + co;
    if (e >= nout) return;
    float s = 0.0f;
    for (int sl = 0; sl < kDwSlices; ++sl) s += red[(long long)sl * nout + e];
    if (e < co * K)
        dW[e] = s;
    else
        db[e - co * K] = s;
}

namespace {
// Position chunks of the weight-gradient reduction: about 1024 positions
// each (enough waves to fill the chip at 1025^2 grids), at least 64.
void dw_split(long long P, int& nchunks, long long& clen)
{
    clen = 1024;
    if (P < 64LL * 1024) clen = (P + 63) / 64;
    clen = (clen + 15) / 16 * 16;
    if (clen < 64) clen = 64;
    nchunks = (int)((P + clen - 1) / clen);
}
}  // namespace

long long cnn_dw_part_floats(long long positions, int cin_pad)
{
    int nchunks;
    long long clen;
    dw_split(positions, nchunks, clen);
    // partials, bias partials, and the stage-1 slices (at most 32 x (32 x 9 x 32 + 32) outputs)
    return (long long)nchunks * ((9 * cin_pad + 31) / 32) * 1024 + (long long)nchunks * 32 +
           (long long)kDwSlices * (32 * 9 * cin_pad + 32);
}

hipError_t cnn_conv_dw(const uint16_t* in, int ci, int cin_pad, int B, int H, int W, const uint16_t* dZ, int co,
                       int cout_pad, float* part, float* dW, float* db, hipStream_t s)
{
    const long long P = (long long)B * H * W;
    int nchunks;
    long long clen;
    dw_split(P, nchunks, clen);
    const int K = ci * 9;
    const int ktiles = (9 * cin_pad + 31) / 32;
    const long long waves = (long long)nchunks * ktiles;
    float* dbpart = part + (long long)nchunks * ktiles * 1024;
    hipLaunchKernelGGL(k_conv_dw, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, in, ci, cin_pad, B, H, W,
                       dZ, co, cout_pad, part, dbpart, nchunks, clen);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    float* red = dbpart + (long long)nchunks * 32;
    const int nout = co * K + co;
    hipLaunchKernelGGL(k_dw_reduce1, dim3((nout + 255) / 256, kDwSlices), dim3(256), 0, s, part, dbpart, nchunks,
                       ktiles, co, ci, cin_pad, red);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dw_reduce2, dim3((nout + 255) / 256), dim3(256), 0, s, red, co, ci, dW, db);
    return hipGetLastError();
}

// ------------------------------------------------------------- weights
// Pack FP32 master weights W[co][ci][3][3] into the forward matrix
// Wf[32][9 * cin_pad] (row o, k = tap * cin_pad + c) and the input-gradient
// matrix Wb[32][9 * cout_pad] (row c, k = tap' * cout_pad + o holding the
// flipped kernel W[o][c][2 - dy'][2 - dx']), both BF16, zero padded.
__global__ void k_pack(const float* __restrict__ Wt, int ci, int co, int cin_pad, int cout_pad,
                       uint16_t* __restrict__ Wf, uint16_t* __restrict__ Wb)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int Kp = 9 * cin_pad, Kpb = 9 * cout_pad;
    if (idx < 32 * Kp) {
        const int o = idx / Kp, k = idx - o * Kp;
        const int tap = k / cin_pad, c = k - tap * cin_pad;
        float v = 0.0f;
        if (o < co && c < ci) v = Wt[(o * ci + c) * 9 + tap];
        Wf[idx] = f2bf(v);
    }
    if (Wb && idx < 32 * Kpb) {
        const int c = idx / Kpb, k = idx - c * Kpb;
        const int tap = k / cout_pad, o = k - tap * cout_pad;
        float v = 0.0f;
        if (c < ci && o < co) v = Wt[(o * ci + c) * 9 + (8 - tap)];   // (2-dy)*3 + (2-dx) = 8 - tap
        Wb[idx] = f2bf(v);
    }
}

hipError_t cnn_pack(const float* Wt, int ci, int co, int cin_pad, int cout_pad, uint16_t* Wf, uint16_t* Wb,
                    hipStream_t s)
{
    const int n = 32 * 9 * (cin_pad > cout_pad ? cin_pad : cout_pad);
    hipLaunchKernelGGL(k_pack, dim3((n + 255) / 256), dim3(256), 0, s, Wt, ci, co, cin_pad, cout_pad, Wf, Wb);
    return hipGetLastError();
}

// Adam update of FP32 parameters p with gradients g (bias-corrected).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

hipError_t cnn_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                    float eps, int t, hipStream_t s)
{
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)t)));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// ------------------------------------------------------------- loss
// Number of valid outputs: per-block partial counts, then one block sums them
// in a fixed order and writes 1 / max(count, 1).
__global__ __launch_bounds__(256) void k_count_partial(const uint8_t* __restrict__ valid, long long n,
                                                       unsigned long long* __restrict__ part)
{
    __shared__ unsigned long long sh[256];
    unsigned long long c = 0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        c += valid[i] ? 1ull : 0ull;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_count_final(const unsigned long long* __restrict__ part, int nb,
                                                     float* __restrict__ inv_out)
{
    __shared__ unsigned long long sh[256];
    unsigned long long c = 0;
    for (int i = threadIdx.x; i < nb; i += 256) c += part[i];
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *inv_out = 1.0f / (float)(sh[0] > 0 ? sh[0] : 1ull);
}

hipError_t cnn_count_valid(const uint8_t* valid, long long n, unsigned long long* part, int nb, float* inv_out,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_count_partial, dim3(nb), dim3(256), 0, s, valid, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_final, dim3(1), dim3(256), 0, s, part, nb, inv_out);
    return hipGetLastError();
}

// Positive-weighted BCE on logits over valid points.  Logits, labels and the
// valid mask are NCHW [b][15][HW]; the loss gradient
// dZ = (w y (s - 1) + (1 - y) s) valid / n_valid is written NHWC [b][HW][16]
// (channel 15 = 0); per-block partial losses go to part.
__global__ __launch_bounds__(256) void k_bce(const float* __restrict__ z, const uint8_t* __restrict__ y,
                                             const uint8_t* __restrict__ valid, long long HW, long long n16,
                                             float pos_w, const float* __restrict__ inv_dev,
                                             uint16_t* __restrict__ dz, float* __restrict__ part)
{
    __shared__ float sh[256];
    const float inv_nvalid = *inv_dev;
    float s = 0.0f;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n16; i += (long long)gridDim.x * 256) {
        const int k = (int)(i & 15);
        const long long P = i >> 4;
        float g = 0.0f;
        if (k < kCnnOut) {
            const long long b = P / HW, p = P - b * HW;
            const long long idx = (b * kCnnOut + k) * HW + p;
            if (valid[idx]) {
                const float zi = z[idx];
                const float yi = y[idx] ? 1.0f : 0.0f;
                // log sigmoid(z) and log(1 - sigmoid(z)) without overflow
                const float l1p = log1pf(expf(-fabsf(zi)));
                const float lsp = -(fmaxf(-zi, 0.0f) + l1p);
                const float lsn = -(fmaxf(zi, 0.0f) + l1p);
                s += -(pos_w * yi * lsp + (1.0f - yi) * lsn);
                const float sg = 1.0f / (1.0f + expf(-zi));
                g = (pos_w * yi * (sg - 1.0f) + (1.0f - yi) * sg) * inv_nvalid;
            }
        }
        dz[i] = f2bf(g);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] * inv_nvalid;
}

hipError_t cnn_bce(const float* z, const uint8_t* y, const uint8_t* valid, long long B, long long HW,
                   float pos_w, const float* inv_dev, uint16_t* dz, float* part, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_bce, dim3(nblocks), dim3(256), 0, s, z, y, valid, HW, B * HW * 16, pos_w, inv_dev, dz,
                       part);
    return hipGetLastError();
}

// FP32 NCHW [b][3][HW] -> BF16 NHWC [b][HW][8] (channels 3..7 zero).
__global__ void k_input_bf16(const float* __restrict__ x, long long HW, long long n8, uint16_t* __restrict__ y)
{
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n8; i += (long long)gridDim.x * 256) {
        const int c = (int)(i & 7);
        const long long P = i >> 3;
        float v = 0.0f;
        if (c < kCnnIn) {
            const long long b = P / HW, p = P - b * HW;
            v = x[(b * kCnnIn + c) * HW + p];
        }
        y[i] = f2bf(v);
    }
}

hipError_t cnn_input_bf16(const float* x, long long B, long long HW, uint16_t* y, hipStream_t s)
{
    const long long n8 = B * HW * 8;
    long long b = (n8 + 255) / 256;
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL(k_input_bf16, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, x, HW, n8, y);
    return hipGetLastError();
}

// ---------------------------------------------------- features and labels
// Level-l vertex (i, j) of an image stored at final resolution (stride s):
// c0 = ln(max(I, 0) / N_abs + 1e-4), c1 = min(r_min, 20) / 10,
// c2 = min(n_cross, 4) / 4.
__device__ __forceinline__ void feature_at(const double* img, const RayFeat* feat, long long pix, double nabs,
                                           float& c0, float& c1, float& c2)
{
    const double I = img[pix];
    c0 = (float)::log((I > 0.0 ? I : 0.0) / nabs + 1e-4);
    c1 = 0.0f;
    c2 = 0.0f;
    if (feat) {
        const RayFeat f = feat[pix];
        c1 = fminf(f.rmin, 20.0f) * 0.1f;
        c2 = (float)(f.ncross < 4 ? f.ncross : 4) * 0.25f;
    }
}

__global__ void k_cnn_features(const double* __restrict__ img, const RayFeat* __restrict__ feat, long long nx,
                               int s, int H, int W, double nabs, float* __restrict__ x)
{
    const long long HW = (long long)H * W;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= HW) return;
    const int j = (int)(t / W), i = (int)(t - (long long)j * W);
    float c0, c1, c2;
    feature_at(img, feat, (long long)j * s * nx + (long long)i * s, nabs, c0, c1, c2);
    x[t] = c0;
    x[HW + t] = c1;
    x[2 * HW + t] = c2;
}

hipError_t cnn_features(const double* img, const RayFeat* feat, long long nx, int s, int H, int W, double nabs,
                        float* x, hipStream_t st)
{
    const long long HW = (long long)H * W;
    hipLaunchKernelGGL(k_cnn_features, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, st, img, feat, nx, s,
                       H, W, nabs, x);
    return hipGetLastError();
}

// Batched form: grid.y = image; N_abs = the image's level-0 normalisation.
// Output either FP32 NCHW x[b][3][H][W] or, if x is null, the network's BF16
// NHWC input xb[b][H][W][8] (channels 3..7 zero; the rounding of
// k_input_bf16, so both routes give the same network input).
__global__ void k_cnn_features_batch(const ImageDesc* __restrict__ desc, const Counters* __restrict__ ctr,
                                     int l, int H, int W, float* __restrict__ x, uint16_t* __restrict__ xb,
                                     const int* __restrict__ imap)
{
    const int b = blockIdx.y;
    const int img = imap ? imap[b] : b;
    const int HW = H * W;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= HW) return;
    const ImageDesc& D = desc[img];
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    // an image of the batch with fewer levels has no level-l grid and the
    // network's output for it is not read; its input is zero
    if (D.levels >= l) {
        const int s = 1 << (D.levels - l);
        const int j = t / W, i = t - j * W;
        feature_at(D.img, D.feat, (long long)j * s * D.nx + (long long)i * s, ctr->scal[img][2], c0, c1, c2);
    }
    if (x) {
        float* xo = x + (long long)b * kCnnIn * HW;
        xo[t] = c0;
        xo[HW + t] = c1;
        xo[2 * HW + t] = c2;
    } else {
        const uint32_t w0 = (uint32_t)f2bf(c0) | ((uint32_t)f2bf(c1) << 16);
        const uint32_t w1 = (uint32_t)f2bf(c2);
        *(uint4*)(xb + ((long long)b * HW + t) * 8) = make_uint4(w0, w1, 0u, 0u);
    }
}

hipError_t cnn_features_batch(const ImageDesc* desc, const Counters* ctr, int nimg, int l, int H, int W,
                              float* x, uint16_t* xb, hipStream_t st, const int* imap)
{
    const long long HW = (long long)H * W;
    if (HW >= (1LL << 31) || (!x && !xb)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cnn_features_batch, dim3((unsigned)((HW + 255) / 256), nimg), dim3(256), 0, st, desc, ctr,
                       l, H, W, x, xb, imap);
    return hipGetLastError();
}

// Offsets (dx, dy) of the points a level-l vertex owns: 3 at level l+1 (in
// level-(l+1) units), then 12 at level l+2 (in level-(l+2) units); together
// the new points of the vertex's cell (right and lower edges included).
__constant__ int kOwnDx[kCnnOut] = { 1, 0, 1, 1, 3, 0, 1, 2, 3, 1, 3, 0, 1, 2, 3 };
__constant__ int kOwnDy[kCnnOut] = { 0, 1, 1, 0, 0, 1, 1, 1, 1, 2, 2, 3, 3, 3, 3 };

__device__ __forceinline__ bool owned_point(int k, int i, int j, int l, int N, int nx0, int ny0, long long nx,
                                            long long& pix, int& lev)
{
    const int up = k < 3 ? 1 : 2;
    lev = l + up;
    if (lev > N) return false;
    const int p = (i << up) + kOwnDx[k], q = (j << up) + kOwnDy[k];
    const int nxl = (1 << lev) * (nx0 - 1) + 1, nyl = (1 << lev) * (ny0 - 1) + 1;
    if (p >= nxl || q >= nyl) return false;
    const int sL = 1 << (N - lev);
    pix = (long long)q * sL * nx + (long long)p * sL;
    return true;
}

// Labels of a plain render's level map: lab[k][j][i] = 1 if the point was
// traced at its level; val = 1 if the point exists.
__global__ void k_cnn_labels(const int8_t* __restrict__ level, long long nx, int nx0, int ny0, int N, int l,
                             uint8_t* __restrict__ lab, uint8_t* __restrict__ val)
{
    const int W = (1 << l) * (nx0 - 1) + 1, H = (1 << l) * (ny0 - 1) + 1;
    const long long HW = (long long)H * W;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= HW) return;
    const int j = (int)(t / W), i = (int)(t - (long long)j * W);
    for (int k = 0; k < kCnnOut; ++k) {
        long long pix = 0;
        int lev;
        const bool ok = owned_point(k, i, j, l, N, nx0, ny0, nx, pix, lev);
        val[k * HW + t] = ok ? 1 : 0;
        lab[k * HW + t] = ok && level[pix] == lev ? 1 : 0;
    }
}

hipError_t cnn_labels(const int8_t* level, long long nx, int nx0, int ny0, int N, int l, uint8_t* lab,
                      uint8_t* val, hipStream_t s)
{
    const int W = (1 << l) * (nx0 - 1) + 1, H = (1 << l) * (ny0 - 1) + 1;
    const long long HW = (long long)H * W;
    hipLaunchKernelGGL(k_cnn_labels, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0, s, level, nx, nx0, ny0,
                       N, l, lab, val);
    return hipGetLastError();
}

// Proposals: one thread per vertex of image blockIdx.y, every output of the
// vertex.  The block's level-(l+2) proposals are counted first and reserved in
// the trace list of pass l+1 with one atomic per block and list end (per wave
// and output, the shared list counter serialised the kernel).  A proposal is
// queued at the front of the list when the largest step count of its cell's
// four level-l corners reaches long_steps, else from the back, as the
// estimator queues the points it flags: the long rays of the look-ahead pass
// start first.
constexpr int kProposeThreads = 256;

__global__ __launch_bounds__(kProposeThreads) void k_cnn_propose(const float* __restrict__ logits,
                                                                 const ImageDesc* __restrict__ desc, int l, int H,
                                                                 int W, float z_hi, float z_lo, int all_levels,
                                                                 unsigned long long* __restrict__ list,
                                                                 long long cap, int long_steps,
                                                                 Counters* __restrict__ ctr,
                                                                 const int* __restrict__ imap)
{
    constexpr int kWaves = kProposeThreads / 64;
    __shared__ unsigned s_cnt[2][kWaves];
    __shared__ unsigned s_base[2];
    const int b = blockIdx.y;                 // slot of the logits
    const int img = imap ? imap[b] : b;       // image of the batch
    const ImageDesc& D = desc[img];
    const int HW = H * W;
    const int v = blockIdx.x * kProposeThreads + threadIdx.x;
    // the network decides for this image only where it can look ahead (its
    // level count reaches l + 2) or everywhere with all_levels; an image with
    // one level left keeps the plain criterion (marks left undecided)
    const bool decides = D.levels >= l + 2 || all_levels;
    const int j = v < HW ? v / W : 0, i = v < HW ? v - j * W : 0;
    unsigned app = 0;                         // bit k: level-(l+2) output k proposed
    if (v < HW) {
        for (int k = 0; k < kCnnOut; ++k) {
            long long pix = 0;
            int lev;
            if (!owned_point(k, i, j, l, D.levels, D.nx0, D.ny0, D.nx, pix, lev)) continue;
            const float z = logits[((long long)b * kCnnOut + k) * HW + v];
            int8_t m = kMarkUnset;            // undecided: the criterion decides
            if (decides && z > z_hi) {
                if (k < 3) {
                    m = kMarkPropose;
                } else {
                    m = (int8_t)lev;
                    app |= 1u << k;
                }
            } else if (decides && z < z_lo) {
                m = kMarkSuppress;
            }
            D.level[pix] = m;
        }
    }
    // expected cost of the cell's proposals: its most expensive corner
    bool front = false;
    if (app && D.cost) {
        const int nxl = (1 << l) * (D.nx0 - 1) + 1, nyl = (1 << l) * (D.ny0 - 1) + 1;
        const long long sL = 1LL << (D.levels - l);
        const int i1 = i + 1 < nxl ? i + 1 : i, j1 = j + 1 < nyl ? j + 1 : j;
        const uint16_t c00 = D.cost[(long long)j * sL * D.nx + (long long)i * sL];
        const uint16_t c10 = D.cost[(long long)j * sL * D.nx + (long long)i1 * sL];
        const uint16_t c01 = D.cost[(long long)j1 * sL * D.nx + (long long)i * sL];
        const uint16_t c11 = D.cost[(long long)j1 * sL * D.nx + (long long)i1 * sL];
        const uint16_t ca = c00 > c10 ? c00 : c10, cb = c01 > c11 ? c01 : c11;
        front = (int)(ca > cb ? ca : cb) >= long_steps;
    }
    const unsigned fb = front ? app : 0u, bb = front ? 0u : app;
    const int wave = threadIdx.x >> 6;
    unsigned wf = 0, wb = 0;
    for (int k = 3; k < kCnnOut; ++k) {
        wf += (unsigned)__popcll(__ballot((fb >> k) & 1u));
        wb += (unsigned)__popcll(__ballot((bb >> k) & 1u));
    }
    if (__lane_id() == 0) {
        s_cnt[0][wave] = wf;
        s_cnt[1][wave] = wb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned nf = 0, nb = 0;
        for (int w = 0; w < kWaves; ++w) { nf += s_cnt[0][w]; nb += s_cnt[1][w]; }
        s_base[0] = nf ? atomicAdd(&ctr->count[l + 1], nf) : 0u;
        s_base[1] = nb ? atomicAdd(&ctr->count_back[l + 1], nb) : 0u;
        if (nf + nb) {
            atomicAdd(&ctr->img_traced[img][l + 1], nf + nb);
            atomicAdd(&ctr->judge[img][4], (unsigned long long)(nf + nb));
        }
    }
    __syncthreads();
    if (wf + wb == 0) return;                 // wave-uniform
    unsigned of = s_base[0], ob = s_base[1];
    for (int w = 0; w < wave; ++w) { of += s_cnt[0][w]; ob += s_cnt[1][w]; }
    for (int k = 3; k < kCnnOut; ++k) {
        const unsigned long long mf = __ballot((fb >> k) & 1u), mb = __ballot((bb >> k) & 1u);
        if ((app >> k) & 1u) {
            long long pix = 0;
            int lev;
            owned_point(k, i, j, l, D.levels, D.nx0, D.ny0, D.nx, pix, lev);
            const unsigned long long item = make_item((uint32_t)img, (uint32_t)pix);
            if (front)
                list[of + __builtin_amdgcn_mbcnt_hi((unsigned)(mf >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mf, 0u))]
                    = item;
            else
                list[cap - 1 - (long long)(ob + __builtin_amdgcn_mbcnt_hi((unsigned)(mb >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((unsigned)mb, 0u)))]
                    = item;
        }
        of += (unsigned)__popcll(mf);
        ob += (unsigned)__popcll(mb);
    }
}

hipError_t cnn_propose(const float* logits, const ImageDesc* desc, int nimg, int l, int H, int W, float z_hi,
                       float z_lo, int all_levels, unsigned long long* list, long long cap, int long_steps,
                       Counters* ctr, hipStream_t s, const int* imap)
{
    const long long HW = (long long)H * W;
    if (HW >= (1LL << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cnn_propose, dim3((unsigned)((HW + kProposeThreads - 1) / kProposeThreads), nimg),
                       dim3(kProposeThreads), 0, s, logits, desc, l, H, W, z_hi, z_lo, all_levels, list, cap,
                       long_steps, ctr, imap);
    return hipGetLastError();
}

}  // namespace art
