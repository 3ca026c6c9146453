// Kernels of the warm-start network: 3x3 convolutions on BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation) for the forward pass and
// both backward passes, and the small elementwise / reduction kernels around
// them (pooling, upsampling, skip add, ReLU backward, MSE loss, Adam).
//
// Tensors are NHWC, channels padded to a multiple of 32 and contiguous, in
// bfloat16 (activations, their gradients, weight copies) or float32 (master
// weights, weight gradients, optimiser moments, the network output).
// Convolution geometry matches the channel domain: periodic in x (the
// channel is periodic), zero padding in y (walls).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "nn_internal.h"

namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float b2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f2b(float f) {
    // round to nearest even (finite inputs)
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
    const uint4 v = *(const uint4*)p;
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// ---------------------------------------------------------------------------
// Convolution as an implicit GEMM: M = output pixels, N = output channels,
// K = 9 taps x input channels.  Each wave owns one 64-pixel row segment
// (four 16-pixel M tiles) and all NT x 16 output channels; a work-group is
// four consecutive segments.  Per K step of 32 channels a wave loads four A
// fragments (16 pixels x 32 channels of the tap's neighbour row, 16 bytes per
// lane) and NT B fragments (weights [co][tap][ci]); each B fragment feeds
// four MFMAs.
//
// MFMA 16x16x32 operand layout: lane l supplies row (A) / column (B) l % 16
// and K elements 8 (l / 16) .. 8 (l / 16) + 7; the result holds column l % 16,
// rows 4 (l / 16) .. 4 (l / 16) + 3.
template <int NT>
__global__ __launch_bounds__(256) void conv_fwd_kernel(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int segs = a.w >> 6;
    const long long nseg = (long long)a.n * a.h * segs;
    const long long sg = (long long)blockIdx.x * 4 + wave;
    if (sg >= nseg) return;
    const int seg = (int)(sg % segs);
    const int row = (int)(sg / segs);            // n * h + y
    const int y = row % a.h;
    const int kq = lane >> 4, li = lane & 15;
    const int x0 = seg << 6;
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ci = a.ci;
    for (int t = 0; t < 9; ++t) {
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        const int yy = y + dy;
        const bool inb = yy >= 0 && yy < a.h;
        const size_t rbase = (size_t)(inb ? row + dy : row) * a.w;
        const uint16_t* xa[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int xx = x0 + 16 * m + li + dx;
            xx = xx < 0 ? xx + a.w : (xx >= a.w ? xx - a.w : xx);
            xa[m] = a.x + (rbase + xx) * ci + 8 * kq;
        }
        const uint16_t* wb = a.wt + ((size_t)li * 9 + t) * ci + 8 * kq;
        for (int c0 = 0; c0 < ci; c0 += 32) {
            bf16x8 av[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) av[m] = inb ? load8(xa[m] + c0) : zero8();
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const bf16x8 bv = load8(wb + (size_t)j * 16 * 9 * ci + c0);
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[m][j], 0, 0, 0);
            }
        }
    }
    // epilogue: lane holds output channel 16 j + li for pixels 16 m + 4 kq + r
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = 16 * j + li;
        const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const size_t pix0 = (size_t)row * a.w + x0 + 16 * m + 4 * kq;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[m][j][r] + bias;
                if (a.relu) v = v > 0.f ? v : 0.f;
                const size_t p = pix0 + r;
                if (a.y16) a.y16[p * a.co + co] = f2b(v);
                if (a.y32 && co < a.y32_ch) a.y32[p * a.y32_ch + co] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The same convolution with the input staged in LDS, for rows of w = 64, 128
// or 256 pixels.  A work-group's 256 output pixels are R = 256 / w whole rows
// (global rows row0 .. row0 + R - 1 over n h); every tap of a 32-channel K
// block reads input rows row0 - 1 .. row0 + R, which are staged once per K
// block with 16-byte loads (zeros outside 0 .. n h - 1; a tap that leaves its
// image reads zeros without looking).  Pixel p keeps its 32 channels in 64
// bytes, four 16-byte slots; slot s sits at s ^ ((p >> 2) & 3), so the 16
// lanes of a fragment (16 consecutive pixels, one slot) hit distinct banks.
// Weight fragments still come through L1: they are the same for every
// work-group.  Per K block the taps run in order 0 .. 8.  LDS is sized at
// launch: (R + 2) w pixels of 64 bytes, 24, 32 or 48 KB for w = 64, 128, 256.
template <int NT>
__global__ __launch_bounds__(256) void conv_fwd_lds_kernel(ConvArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint16_t s_x[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w = a.w, lw = 31 - __clz(w), segs = w >> 6, R = 4 / segs;
    const long long nrows = (long long)a.n * a.h;
    const long long row0 = (long long)blockIdx.x * R;
    const int lr0 = wave / segs;                 // this wave's output row within the group
    const long long row = row0 + lr0;
    const bool active = row < nrows;
    const int y = (int)(row % a.h);
    const int kq = lane >> 4, li = lane & 15;
    const int x0 = (wave - lr0 * segs) << 6;
    const int ci = a.ci;
    const int npieces = (R + 2) * w * 4;         // 16-byte pieces staged per K block
    f32x4 acc[4][NT];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < ci; c0 += 32) {
        __syncthreads();                         // the previous block's reads are done
        for (int q = threadIdx.x; q < npieces; q += 256) {
            const int p = q >> 2, s = q & 3;
            const int lr = p >> lw, col = p & (w - 1);
            const long long grow = row0 - 1 + lr;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (grow >= 0 && grow < nrows) v = *(const uint4*)(a.x + ((size_t)grow * w + col) * ci + c0 + 8 * s);
            *(uint4*)(s_x + p * 32 + 8 * (s ^ ((p >> 2) & 3))) = v;
        }
        __syncthreads();
        if (active) {
#pragma unroll 3
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3 - 1, dx = t % 3 - 1;
                const bool inb = y + dy >= 0 && y + dy < a.h;
                const int lrow = (lr0 + dy + 1) << lw;
                bf16x8 av[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int p = lrow + ((x0 + 16 * m + li + dx) & (w - 1));
                    av[m] = inb ? __builtin_bit_cast(bf16x8, *(const uint4*)(s_x + p * 32 + 8 * (kq ^ ((p >> 2) & 3))))
                                : zero8();
                }
                const uint16_t* wb = a.wt + ((size_t)li * 9 + t) * ci + c0 + 8 * kq;
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const bf16x8 bv = load8(wb + (size_t)j * 16 * 9 * ci);
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[m][j], 0, 0, 0);
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = 16 * j + li;
        const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const size_t pix0 = (size_t)row * w + x0 + 16 * m + 4 * kq;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[m][j][r] + bias;
                if (a.relu) v = v > 0.f ? v : 0.f;
                const size_t p = pix0 + r;
                if (a.y16) a.y16[p * a.co + co] = f2b(v);
                if (a.y32 && co < a.y32_ch) a.y32[p * a.y32_ch + co] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Row-walking convolution for rows of W = 256, 128 or 64 pixels.  A
// work-group walks down RS consecutive steps of one image; a step is the
// R = 256 / W output rows that its 256 pixels cover.  The work-group
// computes CO / SPLIT of the output channels (slice blockIdx.y); per step
// each wave owns 64 pixels of one row and CO / (SPLIT NG) of those channels
// (NG channel groups of waves, 256 NG threads).
//   - The weights of the work-group's channel slice, all 9 taps and CI input
//     channels, are staged in LDS once, in MFMA fragment order (fragment
//     (tap, K block, N tile) is 64 x 16 bytes, lane-contiguous), so a B
//     fragment is one conflict-free 16-byte read.
//   - The R + 2 input rows of a step sit in an LDS ring of R + 2 row slots
//     (slot of image row r: (r + 1) mod (R + 2); rows outside the image are
//     zeros, so taps need no bounds test).  Consecutive steps share two rows:
//     while a step computes, the R rows the next step adds are loaded into
//     registers, and they replace the R rows it drops after the step.
//   - Pixel p of a row keeps each 32-channel K block in 64 bytes, four
//     16-byte pieces; piece s sits at s ^ ((p >> 2) & 3), so the 16 lanes of
//     an A fragment (16 consecutive pixels, one piece) hit distinct banks.
// Arithmetic per output is the same as in the kernels above: bf16 products
// summed in float32 over the 9 taps in order, K block by K block.
template <int CI, int CO, int W, int NG, int SPLIT>
__global__ __launch_bounds__(256 * NG) void conv_fwd_walk_kernel(ConvArgs a, int rs) {
    constexpr int NTH = 256 * NG;
    constexpr int CB = CI / 32;                  // K blocks of 32 channels
    constexpr int COW = CO / SPLIT;              // output channels of this work-group
    constexpr int NTT = COW / 16;                // N tiles of the work-group
    constexpr int NT = NTT / NG;                 // N tiles of a wave
    constexpr int R = 256 / W;                   // output rows per step
    constexpr int NS = R + 2;                    // ring slots (input rows of a step)
    constexpr int SLOT = CB * W * 4;             // 16-byte pieces per row slot
    constexpr int NWF = 9 * CB * NTT * 64;       // 16-byte pieces of weights
    constexpr int NPF = R * SLOT / NTH;          // prefetched pieces per thread
    static_assert((R * SLOT) % NTH == 0 && NT * NG == NTT && COW % 16 == 0, "shape");
    __shared__ uint4 s_w[NWF];
    __shared__ uint4 s_x[NS * SLOT];
    const int co0 = blockIdx.y * COW;            // first output channel of the slice
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wp = wave & 3, grp = wave >> 2;    // pixel quarter, channel group
    const int kq = lane >> 4, li = lane & 15;
    const int lr = wp / (W / 64);                // output row of this wave within a step
    const int x0 = (wp % (W / 64)) * 64;
    const int steps_img = a.h / R;
    // consecutive walks share their boundary rows: give each XCD (block b runs
    // on XCD b mod 8) a contiguous run of walks
    const int wk = (gridDim.x % 8 == 0) ? (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3)) : (int)blockIdx.x;
    const long long gs0 = (long long)wk * rs;                  // first global step
    const int img = (int)(gs0 / steps_img), s0 = (int)(gs0 - (long long)img * steps_img);
    const uint16_t* xim = a.x + (size_t)img * a.h * W * CI;

    // weights of the slice: piece (co, t, c8) -> fragment (t, cb = c8 / 4,
    // j = co / 16), lane co % 16 + 16 (c8 % 4), co counted within the slice
    for (int q = tid; q < NWF; q += NTH) {
        const int c8 = q % (CI / 8), rest = q / (CI / 8);
        const int t = rest % 9, co = rest / 9;
        const int cb = c8 >> 2, j = co >> 4;
        s_w[((t * CB + cb) * NTT + j) * 64 + (co & 15) + 16 * (c8 & 3)] =
            *(const uint4*)(a.wt + ((size_t)(co0 + co) * 9 + t) * CI + 8 * c8);
    }
    // piece q of an input row: pixel q / (4 CB), block (q / 4) % CB, piece q % 4
    auto lds_piece = [](int q) {
        const int px = q / (4 * CB), cb = (q >> 2) % CB, s = q & 3;
        return (cb * W + px) * 4 + (s ^ ((px >> 2) & 3));
    };
    auto load_piece = [&](int row, int q) -> uint4 {
        if (row < 0 || row >= a.h) return make_uint4(0u, 0u, 0u, 0u);
        return *(const uint4*)(xim + ((size_t)row * W) * CI + 8 * q);   // q indexes 8-channel pieces in order
    };
    // first window: rows s0 R - 1 .. s0 R + R
    for (int q = tid; q < NS * SLOT; q += NTH) {
        const int k = q / SLOT, qq = q - k * SLOT;
        const int row = s0 * R - 1 + k;
        s_x[((row + 1) % NS) * SLOT + lds_piece(qq)] = load_piece(row, qq);
    }
    __syncthreads();

    for (int st = 0; st < rs; ++st) {
        const int s = s0 + st;
        // prefetch the R rows the next step adds: s R + R + 1 .. s R + 2 R
        uint4 pf[NPF];
        if (st + 1 < rs) {
#pragma unroll
            for (int k = 0; k < NPF; ++k) {
                const int q = tid + k * NTH, rr = q / SLOT;
                pf[k] = load_piece(s * R + R + 1 + rr, q - rr * SLOT);
            }
        }
        f32x4 acc[4][NT];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3 - 1, dx = t % 3 - 1;
                const int row = s * R + lr + dy;
                const uint4* xs = s_x + ((row + 1) % NS) * SLOT + cb * W * 4;
                bf16x8 av[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int p = (x0 + 16 * m + li + dx) & (W - 1);
                    av[m] = __builtin_bit_cast(bf16x8, xs[p * 4 + (kq ^ ((p >> 2) & 3))]);
                }
                const uint4* ws = s_w + ((t * CB + cb) * NTT + grp * NT) * 64 + lane;
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, ws[j * 64]);
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[m][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv, acc[m][j], 0, 0, 0);
                }
            }
        }
        // epilogue: lane holds output channel co0 + 16 (grp NT + j) + li for pixels 16 m + 4 kq + r
        const size_t prow = ((size_t)img * a.h + (size_t)s * R + lr) * W;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int co = co0 + 16 * (grp * NT + j) + li;
            const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const size_t pix0 = prow + x0 + 16 * m + 4 * kq;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[m][j][r] + bias;
                    if (a.relu) v = v > 0.f ? v : 0.f;
                    const size_t p = pix0 + r;
                    if (a.y16) a.y16[p * CO + co] = f2b(v);
                    if (a.y32 && co < a.y32_ch) a.y32[p * a.y32_ch + co] = v;
                }
            }
        }
        if (st + 1 < rs) {
            __syncthreads();                     // every wave is done with the rows dropped now
#pragma unroll
            for (int k = 0; k < NPF; ++k) {
                const int q = tid + k * NTH, rr = q / SLOT;
                const int row = s * R + R + 1 + rr;
                s_x[((row + 1) % NS) * SLOT + lds_piece(q - rr * SLOT)] = pf[k];
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

// ---------------------------------------------------------------------------
// Weight gradient dW[co][t][ci] = sum_p dY[p][co] X[nbr(p, t)][ci] and bias
// gradient, split over pixel chunks (multiples of 256 pixels).  Block
// (chunk, dy) covers the three taps of one neighbour row as a GEMM with
// M = output channels, N = (tap, 16-channel input group) columns, K =
// pixels.  It walks its chunk in steps of P pixels (128 or 64, dividing the
// row width, so a step never leaves its row); per step dY and the input row
// at x shifts -1, 0, +1 are staged in LDS transposed to [channel][pixel], so
// that MFMA fragments (8 consecutive pixels of one channel) are single
// 16-byte reads.  Staging is at most one item per thread: Q pixels (4 or 8)
// by 8 channels, 16-byte loads of the item's Q dY pixels or of the Q + 2
// input pixels it needs at the three shifts, transposed in registers with
// byte permutes and written as 8- or 16-byte LDS stores; the next step's
// loads are issued before the current step's MFMAs.  Wave w owns the GEMM
// columns w, w + 4, ... for every output-channel tile: per 32-pixel half
// step it reads the dY fragments once and each input fragment once for all
// output tiles.  Partial sums go to work[chunk][co][9][ci] (and
// work_b[chunk][co]); a second kernel adds the chunks in a fixed order.
// Bias gradient (dy = 0 blocks): each dY thread sums its item's pixels over
// the chunk's steps, and the items are added in order at the end.
template <int CO, int CI, int P>
__global__ __launch_bounds__(256) void conv_wgrad2_kernel(WgradArgs a) {
    constexpr int MT = CO / 16, NJ = CI / 16, NCOL = 3 * NJ, MAXC = (NCOL + 3) / 4;
    constexpr int LP = P + 8;                    // LDS row stride (bf16), 16-byte multiple
    // staging item: Q pixels by 8 channels; quartets where they give every
    // thread an item, else octets
    constexpr int Q = ((P / 4) * ((CO + CI) / 8) <= 256) ? 4 : 8;
    constexpr int NOCT = P / Q;                  // pixel groups per step
    constexpr int NYI = NOCT * (CO / 8), NXI = NOCT * (CI / 8);
    static_assert(NYI + NXI <= 256, "one staging item per thread");
    __shared__ __attribute__((aligned(16))) uint16_t s_dy[CO * LP];
    __shared__ __attribute__((aligned(16))) uint16_t s_x[3 * CI * LP];
    // The three blocks of a chunk (dy = -1, 0, 1) read the same dY and
    // overlapping input rows: they run back to back on one XCD (block b goes
    // to XCD b mod 8), so that two of the three reads of each line hit its L2.
    int chunk, dyi;
    {
        const int b = blockIdx.x;
        if (gridDim.x % 24 == 0) {
            const int k = b >> 3;
            chunk = (b & 7) + 8 * (k / 3);
            dyi = k % 3;
        } else {
            chunk = b / 3;
            dyi = b % 3;
        }
    }
    const int dy = dyi - 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = lane >> 4, li = lane & 15;
    // staging items go to the highest threads: the low waves own the extra
    // GEMM columns when the columns do not divide evenly over the waves
    const int sit = 255 - tid;
    const bool is_y = sit < NYI, is_x = !is_y && sit < NYI + NXI;
    const int item = is_y ? sit : (is_x ? sit - NYI : 0);
    const int oct = item % NOCT, grp = item / NOCT;          // pixel group, 8-channel group
    const bool want_b = a.db != nullptr && dy == 0;
    f32x4 acc[MAXC][MT];
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[c][m] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bpart[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) bpart[c] = 0.f;
    const long long p_begin = (long long)chunk * a.chunk_pix;
    const long long p_end = min(p_begin + a.chunk_pix, a.npix);
    const int nst = (int)((p_end - p_begin) / P);
    uint4 ld[Q + 2];
    auto issue = [&](int k) {
        const long long p0 = p_begin + (long long)P * min(k, nst - 1);
        const long long rowp = p0 / a.w;         // n * h + y
        const int x0 = (int)(p0 - rowp * a.w);
        if (is_y) {
#pragma unroll
            for (int q = 0; q < Q; ++q) ld[q] = *(const uint4*)(a.dy + (size_t)(p0 + Q * oct + q) * CO + 8 * grp);
        } else if (is_x) {
            const int y = (int)(rowp % a.h);
            const bool inb = y + dy >= 0 && y + dy < a.h;
            const size_t xrow = (size_t)(inb ? rowp + dy : rowp) * a.w;
#pragma unroll
            for (int q = 0; q < Q + 2; ++q) {
                int xx = x0 + Q * oct - 1 + q;
                xx = xx < 0 ? xx + a.w : (xx >= a.w ? xx - a.w : xx);
                const uint4 v = *(const uint4*)(a.x + (xrow + xx) * CI + 8 * grp);
                ld[q] = inb ? v : make_uint4(0u, 0u, 0u, 0u);
            }
        }
    };
    // transposes with byte permutes: word (lo, hi) = half c & 1 of dword
    // c >> 1 of pixel lo and of pixel hi
    auto word = [](const uint4& lo, const uint4& hi, int c) -> uint32_t {
        const uint32_t a = ((const uint32_t*)&lo)[c >> 1], b = ((const uint32_t*)&hi)[c >> 1];
        return __builtin_amdgcn_perm(b, a, (c & 1) ? 0x07060302u : 0x05040100u);
    };
    // Q / 2 words of a channel row into LDS: 16-byte stores for octets, 8-byte for quartets
    auto put = [](uint16_t* dst, const uint32_t* w) {
        if constexpr (Q == 8) *(uint4*)dst = make_uint4(w[0], w[1], w[2], w[3]);
        else *(uint2*)dst = make_uint2(w[0], w[1]);
    };
    auto stage = [&]() {
        if (is_y) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                uint32_t w[Q / 2];
#pragma unroll
                for (int k = 0; k < Q / 2; ++k) w[k] = word(ld[2 * k], ld[2 * k + 1], c);
                put(&s_dy[(8 * grp + c) * LP + Q * oct], w);
                if (want_b) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) bpart[c] += b2f(((const uint16_t*)&ld[q])[c]);
                }
            }
        } else if (is_x) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                // ld[q] holds pixel Q oct - 1 + q; copy d holds pixel j + d - 1 at position j
                uint32_t ev[Q / 2 + 1], od[Q / 2];   // words (2k, 2k+1) and (2k+1, 2k+2) of the Q + 2 pixels
#pragma unroll
                for (int k = 0; k <= Q / 2; ++k) ev[k] = word(ld[2 * k], ld[2 * k + 1], c);
#pragma unroll
                for (int k = 0; k < Q / 2; ++k) od[k] = word(ld[2 * k + 1], ld[2 * k + 2], c);
                put(&s_x[(0 * CI + 8 * grp + c) * LP + Q * oct], ev);
                put(&s_x[(1 * CI + 8 * grp + c) * LP + Q * oct], od);
                put(&s_x[(2 * CI + 8 * grp + c) * LP + Q * oct], ev + 1);
            }
        }
    };
    issue(0);
    for (int k = 0; k < nst; ++k) {
        stage();
        issue(k + 1);                            // past the last step: reloads it, unused
        __syncthreads();
#pragma unroll
        for (int hf = 0; hf < P / 32; ++hf) {
            bf16x8 af[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) af[m] = load8(&s_dy[(16 * m + li) * LP + 32 * hf + 8 * kq]);
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
                const int col = wave + 4 * c;
                if (col < NCOL) {
                    const int d = col / NJ, nj = col - d * NJ;
                    const bf16x8 bv = load8(&s_x[(d * CI + 16 * nj + li) * LP + 32 * hf + 8 * kq]);
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[c][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m], bv, acc[c][m], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // partials: work[chunk][co][9][ci]
    float* wp = a.work + (size_t)chunk * CO * 9 * CI;
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const int col = wave + 4 * c;
        if (col < NCOL) {
            const int d = col / NJ, nj = col - d * NJ;
            const int t = 3 * (dy + 1) + d;
            const int cin = 16 * nj + li;
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) wp[((size_t)(16 * m + 4 * kq + r) * 9 + t) * CI + cin] = acc[c][m][r];
        }
    }
    if (want_b) {
        // octet partials through LDS (s_dy is free after the last barrier), added in octet order
        float* s_b = (float*)s_dy;               // [grp][oct][8]
        if (is_y) {
#pragma unroll
            for (int c = 0; c < 8; ++c) s_b[(grp * NOCT + oct) * 8 + c] = bpart[c];
        }
        __syncthreads();
        if (tid < CO) {
            const int gq = tid >> 3, c = tid & 7;
            float s = 0.f;
            for (int o = 0; o < NOCT; ++o) s += s_b[(gq * NOCT + o) * 8 + c];
            a.work_b[(size_t)chunk * CO + tid] = s;
        }
    }
}

// Fixed-order sum of the weight-gradient chunks.  A block owns 64
// consecutive elements (the weights, then the biases).  Wave q adds the
// chunks of its quarter of the chunk range in four interleaved partial sums
// (independent loads in flight), and the four waves' sums are added in order
// through LDS.
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(WgradArgs a) {
    __shared__ float part[4][64];
    const long long nw = (long long)a.co * 9 * a.ci;
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const long long k = (long long)blockIdx.x * 64 + lane;
    const bool isw = k < nw, isb = !isw && a.db && k < nw + a.co;
    const float* src = isw ? a.work + k : (isb ? a.work_b + (k - nw) : nullptr);
    const size_t stride = isw ? (size_t)nw : (size_t)a.co;
    const int per = (a.n_chunks + 3) / 4, c0 = q * per, c1 = min(a.n_chunks, c0 + per);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (src) {
        int c = c0;
        for (; c + 4 <= c1; c += 4) {
            s0 += src[(size_t)c * stride];
            s1 += src[(size_t)(c + 1) * stride];
            s2 += src[(size_t)(c + 2) * stride];
            s3 += src[(size_t)(c + 3) * stride];
        }
        for (; c < c1; ++c) s0 += src[(size_t)c * stride];
    }
    part[q][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (q == 0 && src) {
        const float t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        if (isw) {
            a.dw[k] = a.accumulate ? a.dw[k] + t : t;
        } else {
            const int cb = (int)(k - nw);
            a.db[cb] = a.accumulate ? a.db[cb] + t : t;
        }
    }
}

// ---------------------------------------------------------------------------
// Elementwise kernels (NHWC bf16).

__global__ __launch_bounds__(256) void relu_bwd_kernel(const uint16_t* dy, const uint16_t* y, uint16_t* dx, long long n) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k < n) dx[k] = b2f(y[k]) > 0.f ? dy[k] : (uint16_t)0;
}

__global__ __launch_bounds__(256) void add_kernel(const uint16_t* a, const uint16_t* b, uint16_t* o, long long n) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k < n) o[k] = f2b(b2f(a[k]) + b2f(b[k]));
}

// Pooling and upsampling move 8 channels (16 bytes) per thread; c is a
// multiple of 8.  blockIdx.y walks output rows (image b, row i), so the
// per-thread index arithmetic is 32-bit and small.  Arithmetic per channel
// is unchanged: the pooled value is 0.25 (x00 + x01 + x10 + x11) in float.
__device__ __forceinline__ uint4 ld16(const uint16_t* p) { return *(const uint4*)p; }
__device__ __forceinline__ void st16(uint16_t* p, uint4 v) { *(uint4*)p = v; }
__device__ __forceinline__ float lo_f(uint32_t v) { return __uint_as_float(v << 16); }
__device__ __forceinline__ float hi_f(uint32_t v) { return __uint_as_float(v & 0xffff0000u); }
__device__ __forceinline__ uint32_t pk(float lo, float hi) { return (uint32_t)f2b(lo) | ((uint32_t)f2b(hi) << 16); }

// average pool 2x2: x [n][h][w][c] -> y [n][h/2][w/2][c]
__global__ __launch_bounds__(256) void pool_fwd_kernel(const uint16_t* x, uint16_t* y, int n, int h, int w, int c) {
    const int cg = c >> 3, ho = h >> 1, wo = w >> 1;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= wo * cg) return;
    const int j = t / cg, g = t - j * cg;
    for (int r = blockIdx.y; r < n * ho; r += gridDim.y) {
        const int b = r / ho, i = r - b * ho;
        const size_t base = (((size_t)b * h + 2 * i) * w + 2 * j) * c + 8 * g;
        const size_t rs = (size_t)w * c;
        const uint4 a = ld16(x + base), bq = ld16(x + base + c), cq = ld16(x + base + rs), d = ld16(x + base + rs + c);
        const uint32_t* A = (const uint32_t*)&a; const uint32_t* B = (const uint32_t*)&bq;
        const uint32_t* C = (const uint32_t*)&cq; const uint32_t* D = (const uint32_t*)&d;
        uint4 o;
        uint32_t* O = (uint32_t*)&o;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float sl = lo_f(A[e]) + lo_f(B[e]) + lo_f(C[e]) + lo_f(D[e]);
            const float sh = hi_f(A[e]) + hi_f(B[e]) + hi_f(C[e]) + hi_f(D[e]);
            O[e] = pk(0.25f * sl, 0.25f * sh);
        }
        st16(y + ((size_t)r * wo + j) * c + 8 * g, o);
    }
}

// adjoint of the pool: dx [n][h][w][c] = 0.25 dy [n][h/2][w/2][c]
__global__ __launch_bounds__(256) void pool_bwd_kernel(const uint16_t* dy, uint16_t* dx, int n, int h, int w, int c) {
    const int cg = c >> 3, ho = h >> 1, wo = w >> 1;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= w * cg) return;
    const int xx = t / cg, g = t - xx * cg;
    for (int r = blockIdx.y; r < n * h; r += gridDim.y) {
        const int b = r / h, yy = r - b * h;
        const uint4 v = ld16(dy + (((size_t)b * ho + (yy >> 1)) * wo + (xx >> 1)) * c + 8 * g);
        const uint32_t* V = (const uint32_t*)&v;
        uint4 o;
        uint32_t* O = (uint32_t*)&o;
#pragma unroll
        for (int e = 0; e < 4; ++e) O[e] = pk(0.25f * lo_f(V[e]), 0.25f * hi_f(V[e]));
        st16(dx + ((size_t)r * w + xx) * c + 8 * g, o);
    }
}

// nearest-neighbour x2 upsampling; (h, w) are the input sizes.
__global__ __launch_bounds__(256) void up_fwd_kernel(const uint16_t* x, uint16_t* y, int n, int h, int w, int c) {
    const int cg = c >> 3, W2 = 2 * w, H2 = 2 * h;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= W2 * cg) return;
    const int xx = t / cg, g = t - xx * cg;
    for (int r = blockIdx.y; r < n * H2; r += gridDim.y) {
        const int b = r / H2, yy = r - b * H2;
        st16(y + ((size_t)r * W2 + xx) * c + 8 * g, ld16(x + (((size_t)b * h + (yy >> 1)) * w + (xx >> 1)) * c + 8 * g));
    }
}

// adjoint of the upsampling: dx [n][h][w][c] = sum of the four dy it fed
__global__ __launch_bounds__(256) void up_bwd_kernel(const uint16_t* dy, uint16_t* dx, int n, int h, int w, int c) {
    const int cg = c >> 3;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= w * cg) return;
    const int j = t / cg, g = t - j * cg;
    for (int r = blockIdx.y; r < n * h; r += gridDim.y) {
        const int b = r / h, i = r - b * h;
        const size_t base = (((size_t)b * 2 * h + 2 * i) * 2 * w + 2 * j) * c + 8 * g;
        const size_t rs = (size_t)2 * w * c;
        const uint4 a = ld16(dy + base), bq = ld16(dy + base + c), cq = ld16(dy + base + rs), d = ld16(dy + base + rs + c);
        const uint32_t* A = (const uint32_t*)&a; const uint32_t* B = (const uint32_t*)&bq;
        const uint32_t* C = (const uint32_t*)&cq; const uint32_t* D = (const uint32_t*)&d;
        uint4 o;
        uint32_t* O = (uint32_t*)&o;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            O[e] = pk(lo_f(A[e]) + lo_f(B[e]) + lo_f(C[e]) + lo_f(D[e]), hi_f(A[e]) + hi_f(B[e]) + hi_f(C[e]) + hi_f(D[e]));
        st16(dx + ((size_t)r * w + j) * c + 8 * g, o);
    }
}

// ReLU backward and the skip add, 8 elements (16 bytes) per thread: used
// when the count is a multiple of 8 and every buffer is 16-byte aligned.
// Per element the result is the scalar kernels' (out may alias an input).
__global__ __launch_bounds__(256) void relu_bwd_vec_kernel(const uint16_t* dy, const uint16_t* y, uint16_t* dx,
                                                           long long n8) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= n8) return;
    const uint4 d = ((const uint4*)dy)[k], v = ((const uint4*)y)[k];
    const uint32_t* D = (const uint32_t*)&d;
    const uint32_t* V = (const uint32_t*)&v;
    uint4 o;
    uint32_t* O = (uint32_t*)&o;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        O[e] = (lo_f(V[e]) > 0.f ? (D[e] & 0xffffu) : 0u) | (hi_f(V[e]) > 0.f ? (D[e] & 0xffff0000u) : 0u);
    ((uint4*)dx)[k] = o;
}

__global__ __launch_bounds__(256) void add_vec_kernel(const uint16_t* a, const uint16_t* b, uint16_t* o, long long n8) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= n8) return;
    const uint4 x = ((const uint4*)a)[k], z = ((const uint4*)b)[k];
    const uint32_t* X = (const uint32_t*)&x;
    const uint32_t* Z = (const uint32_t*)&z;
    uint4 r;
    uint32_t* R = (uint32_t*)&r;
#pragma unroll
    for (int e = 0; e < 4; ++e) R[e] = pk(lo_f(X[e]) + lo_f(Z[e]), hi_f(X[e]) + hi_f(Z[e]));
    ((uint4*)o)[k] = r;
}

// MSE over the nch real output channels: loss = sum (pred - tgt)^2 / (npix nch);
// dpred (bf16, cpad channels, zero beyond nch) = 2 (pred - tgt) / (npix nch).
// Per-block float64 partial sums of the loss go to partial[block].
__global__ __launch_bounds__(256) void mse_kernel(const float* pred, const float* tgt, uint16_t* dpred, double* partial,
                                                  long long npix, int nch, int cpad) {
    __shared__ double s[256];
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (k < npix) {
        const float inv = 1.0f / (float)((double)npix * nch);
        for (int c = 0; c < nch; ++c) {
            const float d = pred[k * nch + c] - tgt[k * nch + c];
            l += (double)d * d;
            if (dpred) dpred[k * cpad + c] = f2b(2.f * d * inv);
        }
        if (dpred)
            for (int c = nch; c < cpad; ++c) dpred[k * cpad + c] = 0;
    }
    s[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void sum_kernel(const double* partial, int n, double scale, double* out) {
    __shared__ double s[256];
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) v += partial[k];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] * scale;
}

// Adam (bias-corrected) on float32 master weights [co][9][ci]; refreshes the
// bf16 copy and the flipped, transposed copy [ci][8 - t][co] that the
// data-gradient convolution uses.  wflip may be null (bias vectors: co = n,
// ci = 1, taps = 1).
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= a.n) return;
    const float g = a.g[k];
    const float m = a.b1 * a.m[k] + (1.f - a.b1) * g;
    const float v = a.b2 * a.v[k] + (1.f - a.b2) * g * g;
    a.m[k] = m;
    a.v[k] = v;
    const float mh = m * a.c1, vh = v * a.c2;
    float w = a.w[k];
    w -= a.lr * (mh / (sqrtf(vh) + a.eps) + a.wd * w);
    a.w[k] = w;
    const uint16_t wb = f2b(w);
    if (a.w16) a.w16[k] = wb;
    if (a.wflip) {
        const int ci = (int)(k % a.ci);
        const long long q = k / a.ci;
        const int t = (int)(q % 9);
        const int co = (int)(q / 9);
        a.wflip[((size_t)ci * 9 + (8 - t)) * a.co + co] = wb;
    }
}

// float32 master weights -> bf16 copy and flipped copy (set-up, no update)
__global__ __launch_bounds__(256) void wcast_kernel(const float* w, uint16_t* w16, uint16_t* wflip, int co, int ci) {
    const long long n = (long long)co * 9 * ci;
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const uint16_t wb = f2b(w[k]);
    w16[k] = wb;
    if (wflip) {
        const int c = (int)(k % ci);
        const long long q = k / ci;
        const int t = (int)(q % 9);
        const int o = (int)(q / 9);
        wflip[((size_t)c * 9 + (8 - t)) * co + o] = wb;
    }
}

// ---------------------------------------------------------------------------
// Channel features and the hand-off to the LBM.

__device__ __forceinline__ double phi_tanh(const ChanDesc& d, int j) {
    return 0.5 * (1.0 + tanh(2.0 * ((d.b - 0.5) - (double)j) / d.W));
}

// x[n][y][x][cpad]: the 8 input planes of channel n (the rest zero).
__global__ __launch_bounds__(256) void features_kernel(const ChanDesc* desc, uint16_t* x, int n, int h, int w, int cpad) {
    const long long total = (long long)n * h * w;
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= total) return;
    const int i = (int)(k % w);
    const int j = (int)((k / w) % h);
    const int b = (int)(k / ((long long)w * h));
    const ChanDesc& d = desc[b];
    const double ph = phi_tanh(d, j);
    float f[NFEAT];
    f[0] = (float)(d.dT * cos(2.0 * 3.14159265358979323846 * (double)i / d.l) + (d.T_h - d.T_ref));
    f[1] = (float)ph;
    f[2] = (float)((d.mu_a + ph * (d.mu_b - d.mu_a)) / d.mu_b);
    f[3] = (float)((d.k_a + ph * (d.k_b - d.k_a)) / d.k_b);
    f[4] = (float)(d.sigma_T / 2e-4);
    f[5] = (float)(d.sigma_TT / 3e-4);
    f[6] = (float)(((double)j + 0.5) / h);
    f[7] = (float)(d.b / h);
    f[8] = (float)(log(d.mu_a / d.mu_b) / log(5.0));
    f[9] = (float)(log(d.k_a / d.k_b) / log(5.0));
    uint16_t* o = x + (size_t)k * cpad;
    for (int c = 0; c < cpad; ++c) o[c] = c < NFEAT ? f2b(f[c]) : (uint16_t)0;
}

// pred[n][y][x][4] (u / U_s, v / U_s, (T - T_ref) / dT, phi) -> LBM init fields
// [n][phi | ux | uy | T][y][x] in float64.  phi: the network's, clipped to
// [0, 1] (phi_net != 0), or the cold-start tanh profile.
__device__ __forceinline__ bool in_band(const ChanDesc& d, int j) {
    return fabs((double)j - (d.b - 0.5)) <= PHI_BAND * d.W;
}
// shape of a rigid shift of the cold-start interface (proportional to its
// y-derivative)
__device__ __forceinline__ double shift_shape(const ChanDesc& d, int j) {
    const double c = cosh(2.0 * ((d.b - 0.5) - (double)j) / d.W);
    return 1.0 / (c * c);
}

// One block per channel.  phi: the cold-start profile, plus (phi_net) the
// predicted deviation on the interface band and the rigid interface shift
// that returns sum phi to the cold start's (sum over the band of the
// deviation, S, cancelled by -S / (w sum_j g(j)) g(j)).
__global__ __launch_bounds__(256) void to_fields_kernel(const ChanDesc* desc, const float* pred, double* fields, int h, int w,
                                                        int phi_net) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    const ChanDesc& d = desc[b];
    const long long hw = (long long)h * w;
    const float* P = pred + (size_t)b * hw * 4;
    double* o = fields + (size_t)b * 4 * hw;
    double corr = 0.0;
    if (phi_net) {
        double s = 0.0;
        for (long long q = threadIdx.x; q < hw; q += 256)
            if (in_band(d, (int)(q / w))) s += (double)P[q * 4 + 3];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        double G = 0.0;
        for (int j = 0; j < h; ++j)
            if (in_band(d, j)) G += shift_shape(d, j);
        corr = G > 0.0 ? -(red[0] / PHI_DEV_SCALE) / (G * (double)w) : 0.0;
    }
    for (long long q = threadIdx.x; q < hw; q += 256) {
        const int j = (int)(q / w);
        const float* p = P + q * 4;
        double ph = phi_tanh(d, j);
        if (phi_net && in_band(d, j)) ph += (double)p[3] / PHI_DEV_SCALE + corr * shift_shape(d, j);
        o[q] = ph;
        o[hw + q] = (double)p[0] * d.U_s;
        o[2 * hw + q] = (double)p[1] * d.U_s;
        o[3 * hw + q] = d.T_ref + d.dT * (double)p[2];
    }
}

// converged LBM fields [n][phi | ux | uy | T][y][x] float64 -> targets [n][y][x][4] float32
__global__ __launch_bounds__(256) void targets_kernel(const ChanDesc* desc, const double* fields, float* tgt, int n, int h, int w) {
    const long long total = (long long)n * h * w;
    const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
    if (k >= total) return;
    const long long hw = (long long)h * w;
    const int b = (int)(k / hw);
    const long long q = k - b * hw;
    const ChanDesc& d = desc[b];
    const double* f = fields + (size_t)b * 4 * hw;
    float* o = tgt + (size_t)k * 4;
    o[0] = (float)(f[hw + q] / d.U_s);
    o[1] = (float)(f[2 * hw + q] / d.U_s);
    o[2] = (float)((f[3 * hw + q] - d.T_ref) / d.dT);
    const int j = (int)(q / w);
    o[3] = in_band(d, j) ? (float)((f[q] - phi_tanh(d, j)) * PHI_DEV_SCALE) : 0.0f;
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_of(long long n) { return (unsigned)((n + 255) / 256); }
static inline bool al16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Steps per work-group of the row-walking kernel: fixed by nn_set_conv_walk
// (tests, tuning), else the largest of 8, 4, 2 that divides the steps of an
// image and still leaves one round of work-groups, as many as the CUs hold
// at once (256 CUs times the work-groups that fit on one CU, from the
// runtime's occupancy query: LDS and registers), else 1.  Longer walks share
// more input rows and stage the weights fewer times.
static int g_walk_rs = 0;

static int walk_steps(int steps_img, long long groups, int per_cu) {
    if (g_walk_rs > 0) return (steps_img % g_walk_rs == 0) ? g_walk_rs : 1;
    for (int rs = 8; rs >= 2; rs >>= 1)
        if (steps_img % rs == 0 && groups / rs >= 256LL * per_cu) return rs;
    return 1;
}

template <int CI, int CO, int W, int NG, int SPLIT = 1>
static hipError_t walk_launch(const ConvArgs& a, hipStream_t st) {
    constexpr int R = 256 / W;
    static int per_cu = 0;                       // resident work-groups per CU, queried once
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_fwd_walk_kernel<CI, CO, W, NG, SPLIT>, 256 * NG, 0) !=
                hipSuccess || nb < 1)
            nb = 1;
        per_cu = nb;
    }
    const int steps_img = a.h / R;
    const long long total = (long long)a.n * steps_img;
    const int rs = walk_steps(steps_img, total * SPLIT, per_cu);
    conv_fwd_walk_kernel<CI, CO, W, NG, SPLIT><<<dim3((unsigned)(total / rs), SPLIT), 256 * NG, 0, st>>>(a, rs);
    return hipGetLastError();
}

// Row-walking kernel where it is compiled: rows of 256, 128 or 64 pixels,
// whole steps per image, the channel pairs of the network's layers.  The
// unsplit layers run 512-thread work-groups of two channel groups (measured
// 2-10% faster than one group for the 32-channel outputs at batch 32); the
// 96-channel pairs split their output channels over two work-groups so that
// their weights fit in LDS beside the input rows.  Other shapes take the
// LDS-staged kernel for rows of 64, 128 or 256 pixels, except with 32 input
// and 32 output channels: there a work-group has one K block, the staging
// latency is exposed, and the unstaged kernel is faster (measured at batch
// 32 on the network's layers: 0.075 against 0.081 ms at 256 x 128; every
// other layer is 15-45% faster staged).
hipError_t launch_conv_fwd(const ConvArgs& a, hipStream_t st) {
    if (a.w == 256) {
        const int key = a.ci * 1000 + a.co;
        switch (key) {
            case 32032: return walk_launch<32, 32, 256, 2>(a, st);
            case 64032: return walk_launch<64, 32, 256, 2>(a, st);
            case 32064: return walk_launch<32, 64, 256, 2>(a, st);
            default: break;
        }
    }
    if (a.w == 128 && a.h % 2 == 0) {
        const int key = a.ci * 1000 + a.co;
        switch (key) {
            case 32064: return walk_launch<32, 64, 128, 2>(a, st);
            case 64032: return walk_launch<64, 32, 128, 2>(a, st);
            case 64064: return walk_launch<64, 64, 128, 2>(a, st);
            case 96064: return walk_launch<96, 64, 128, 1, 2>(a, st);
            case 64096: return walk_launch<64, 96, 128, 1, 2>(a, st);
            default: break;
        }
    }
    if (a.w == 64 && a.h % 4 == 0) {
        const int key = a.ci * 1000 + a.co;
        switch (key) {
            case 64096: return walk_launch<64, 96, 64, 1, 2>(a, st);
            case 96096: return walk_launch<96, 96, 64, 1, 2>(a, st);
            case 96064: return walk_launch<96, 64, 64, 1, 2>(a, st);
            default: break;
        }
    }
    if ((a.w == 64 || a.w == 128 || a.w == 256) && !(a.ci == 32 && a.co == 32)) {
        const int R = 256 / a.w;                 // output rows per work-group
        const unsigned grid = (unsigned)(((long long)a.n * a.h + R - 1) / R);
        const size_t lds = (size_t)(R + 2) * a.w * 64;
        switch (a.co / 16) {
            case 2: conv_fwd_lds_kernel<2><<<grid, 256, lds, st>>>(a); break;
            case 4: conv_fwd_lds_kernel<4><<<grid, 256, lds, st>>>(a); break;
            case 6: conv_fwd_lds_kernel<6><<<grid, 256, lds, st>>>(a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)(((long long)a.n * a.h * (a.w / 64) + 3) / 4);
    switch (a.co / 16) {
        case 2: conv_fwd_kernel<2><<<grid, 256, 0, st>>>(a); break;
        case 4: conv_fwd_kernel<4><<<grid, 256, 0, st>>>(a); break;
        case 6: conv_fwd_kernel<6><<<grid, 256, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Pixels per step of the weight-gradient kernel: 128 where the row width
// allows it and both channel counts are at most 64 (LDS at 70 KB or less),
// else 64.  Measured on the network's layers at batch 32, 128-pixel steps
// beat 64-pixel ones even where they leave fewer blocks per CU (32 x 64:
// 0.187 against 0.232 ms; 64 x 64: 0.063 against 0.089 ms).
// The chunk count is cut, where that helps, to what one round of resident
// blocks covers (three blocks per chunk; 256 CUs times the blocks that fit
// on one, from the runtime's occupancy query), rounded down to a multiple of
// 8: a layer whose blocks do not all fit at once would otherwise run one and
// a half rounds.  Fewer, longer chunks fit in the workspace sized for the
// default count; the sum stays deterministic (a function of the sizes and
// the kernel).
template <int CO, int CI, int P>
static void wgrad2_launch(WgradArgs& a, hipStream_t st) {
    static int per_cu = 0;
    if (per_cu == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_wgrad2_kernel<CO, CI, P>, 256, 0) != hipSuccess ||
            nb < 1)
            nb = 1;
        per_cu = nb;
    }
    const long long want = (256LL * per_cu / 3) / 8 * 8;
    if (want >= 8 && want < a.n_chunks) {
        long long cp = (a.npix + want - 1) / want;
        cp = ((cp + 255) / 256) * 256;
        a.chunk_pix = cp;
        a.n_chunks = (int)((a.npix + cp - 1) / cp);
        a.work_b = a.work + (size_t)a.n_chunks * CO * 9 * CI;
    }
    conv_wgrad2_kernel<CO, CI, P><<<(unsigned)(3 * a.n_chunks), 256, 0, st>>>(a);
}

template <int CO, int CI>
static void wgrad_launch(WgradArgs& a, hipStream_t st) {
    constexpr bool P128 = CO <= 64 && CI <= 64;
    if (P128 && a.w % 128 == 0) wgrad2_launch<CO, CI, P128 ? 128 : 64>(a, st);
    else wgrad2_launch<CO, CI, 64>(a, st);
}

void set_conv_walk(int rs) { g_walk_rs = rs; }

hipError_t launch_conv_wgrad(const WgradArgs& args, hipStream_t st) {
    WgradArgs a = args;                          // the launch may choose longer chunks
    const int key = (a.co / 32) * 4 + a.ci / 32;
    switch (key) {
        case 1 * 4 + 1: wgrad_launch<32, 32>(a, st); break;
        case 1 * 4 + 2: wgrad_launch<32, 64>(a, st); break;
        case 1 * 4 + 3: wgrad_launch<32, 96>(a, st); break;
        case 2 * 4 + 1: wgrad_launch<64, 32>(a, st); break;
        case 2 * 4 + 2: wgrad_launch<64, 64>(a, st); break;
        case 2 * 4 + 3: wgrad_launch<64, 96>(a, st); break;
        case 3 * 4 + 1: wgrad_launch<96, 32>(a, st); break;
        case 3 * 4 + 2: wgrad_launch<96, 64>(a, st); break;
        case 3 * 4 + 3: wgrad_launch<96, 96>(a, st); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    wgrad_reduce_kernel<<<(unsigned)(((long long)a.co * 9 * a.ci + a.co + 63) / 64), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_relu_bwd(const uint16_t* dy, const uint16_t* y, uint16_t* dx, long long n, hipStream_t st) {
    if (n % 8 == 0 && al16(dy) && al16(y) && al16(dx)) relu_bwd_vec_kernel<<<blocks_of(n / 8), 256, 0, st>>>(dy, y, dx, n / 8);
    else relu_bwd_kernel<<<blocks_of(n), 256, 0, st>>>(dy, y, dx, n);
    return hipGetLastError();
}

hipError_t launch_add(const uint16_t* a, const uint16_t* b, uint16_t* o, long long n, hipStream_t st) {
    if (n % 8 == 0 && al16(a) && al16(b) && al16(o)) add_vec_kernel<<<blocks_of(n / 8), 256, 0, st>>>(a, b, o, n / 8);
    else add_kernel<<<blocks_of(n), 256, 0, st>>>(a, b, o, n);
    return hipGetLastError();
}

// grid of the row-wise pooling / upsampling kernels: x covers one output
// row's (pixel, 8-channel group) pairs, y walks the output rows
static dim3 row_grid(long long row_items, long long rows) {
    return dim3((unsigned)((row_items + 255) / 256), (unsigned)std::min<long long>(rows, 65535));
}

hipError_t launch_pool(int dir, const uint16_t* in, uint16_t* out, int n, int h, int w, int c, hipStream_t st) {
    const int cg = c / 8;
    if (dir == 0) pool_fwd_kernel<<<row_grid((long long)(w / 2) * cg, (long long)n * (h / 2)), 256, 0, st>>>(in, out, n, h, w, c);
    else pool_bwd_kernel<<<row_grid((long long)w * cg, (long long)n * h), 256, 0, st>>>(in, out, n, h, w, c);
    return hipGetLastError();
}

hipError_t launch_up(int dir, const uint16_t* in, uint16_t* out, int n, int h, int w, int c, hipStream_t st) {
    const int cg = c / 8;
    if (dir == 0) up_fwd_kernel<<<row_grid((long long)2 * w * cg, (long long)n * 2 * h), 256, 0, st>>>(in, out, n, h, w, c);
    else up_bwd_kernel<<<row_grid((long long)w * cg, (long long)n * h), 256, 0, st>>>(in, out, n, h, w, c);
    return hipGetLastError();
}

hipError_t launch_mse(const float* pred, const float* tgt, uint16_t* dpred, double* partial, double* out,
                      long long npix, int nch, int cpad, hipStream_t st) {
    const unsigned nb = blocks_of(npix);
    mse_kernel<<<nb, 256, 0, st>>>(pred, tgt, dpred, partial, npix, nch, cpad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sum_kernel<<<1, 256, 0, st>>>(partial, (int)nb, 1.0 / ((double)npix * nch), out);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t st) {
    adam_kernel<<<blocks_of(a.n), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_wcast(const float* w, uint16_t* w16, uint16_t* wflip, int co, int ci, hipStream_t st) {
    wcast_kernel<<<blocks_of((long long)co * 9 * ci), 256, 0, st>>>(w, w16, wflip, co, ci);
    return hipGetLastError();
}

hipError_t launch_features(const ChanDesc* d, uint16_t* x, int n, int h, int w, int cpad, hipStream_t st) {
    features_kernel<<<blocks_of((long long)n * h * w), 256, 0, st>>>(d, x, n, h, w, cpad);
    return hipGetLastError();
}

hipError_t launch_to_fields(const ChanDesc* d, const float* pred, double* fields, int n, int h, int w, int phi_net,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    to_fields_kernel<<<(unsigned)n, 256, 0, st>>>(d, pred, fields, h, w, phi_net);
    return hipGetLastError();
}

hipError_t launch_targets(const ChanDesc* d, const double* fields, float* tgt, int n, int h, int w, hipStream_t st) {
    targets_kernel<<<blocks_of((long long)n * h * w), 256, 0, st>>>(d, fields, tgt, n, h, w);
    return hipGetLastError();
}

}  // namespace nn
