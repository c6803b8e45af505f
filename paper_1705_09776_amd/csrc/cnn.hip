// Surrogate candidate-mask CNN on gfx950 (not from the paper: a learned gate
// in front of ALP detection).  Per image at 1/4 resolution:
//   X0 = space-to-depth(4) of u8/255 (edge-padded to a multiple of 4),
//   X_l = relu(conv3x3(X_{l-1})), l = 1..4, 16 -> 16 channels, zero padding,
//   Z = X4 . Wh + bh (16 -> 6, one logit per octave), mask bit o = Z_o > logit(tau).
// Activations are bf16 in HWC order (16 channels = 32 bytes per cell); the
// 3x3 convolutions of the forward pass and of both backward passes are
// v_mfma_f32_16x16x16_bf16 with fp32 accumulation; the head is fp32 VALU.
//
// MFMA 16x16x16 bf16 operand layout (wave64, checked on the device): lane l
// holds A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16] for j = 0..3, and
// D[4(l/16)+r][l%16] for r = 0..3.
//
// Parameter vector (fp32, 9382): for l = 1..4: W_l[9][16][16] ([tap][ci][co],
// tap = 3(dy+1)+(dx+1)) then b_l[16]; then Wh[16][6] ([c][o]) then bh[6].
#include "cdvs_internal.h"

namespace cdvs {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

// Forward 3x3 convolutions use v_mfma_f32_16x16x32_bf16, two taps per
// instruction: lane l holds A[l%16][8(l/16)+j] and B[8(l/16)+j][l%16] for
// j = 0..7 (checked on the device), so with k = 16 (tap - 2m) + ci the lanes
// with l/16 = 2h + c carry tap 2m + h, input channels 8c..8c+7; the tenth tap
// of the last pair is zero.
constexpr int kTapPairs = 5;
__device__ __forceinline__ f4 mfma32(const s8& a, const s8& b, const f4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
}

constexpr int CC = kCnnChannels;   // 16
constexpr int NHD = kCnnHeads;     // 6
constexpr int CONV_W = 9 * CC * CC;
constexpr int LAYER_P = CONV_W + CC;

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf2f(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }
// max(x, 0) as one median (x is finite)
__device__ __forceinline__ float relu(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 3.402823466e38f); }
// Two floats -> two bf16 in one word (low half: a), by the hardware
// conversion, which rounds to nearest even as f2bf does (finite inputs).
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){a, b}, bf2v));
}

__device__ __forceinline__ int find_cnn_image(const CnnImage* im, int n, int tile) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (im[mid].tile0 <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_cell_image(const CnnImage* im, int n, int64_t cell) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (im[mid].cell0 <= cell) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Four consecutive s2d channels ci = 4 kb + j (row kb of the 4x4 block,
// columns j = 0..3) of cell (cy, cx), as bf16: u8/255 with edge clamping.
__device__ __forceinline__ s4 s2d_frag(const uint8_t* __restrict__ images, const CnnImage& g, int cy, int cx,
                                       int kb) {
    const int y = min(4 * cy + kb, g.H - 1);
    const uint8_t* row = images + g.src + (int64_t)y * g.src_pitch;
    s4 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = f2bf((float)row[min(4 * cx + j, g.W - 1)] / 255.f);
    return b;
}

// One s2d channel ci of cell (cy, cx).
__device__ __forceinline__ short s2d_chan(const uint8_t* __restrict__ images, const CnnImage& g, int cy, int cx,
                                          int ci) {
    const int y = min(4 * cy + (ci >> 2), g.H - 1), x = min(4 * cx + (ci & 3), g.W - 1);
    return f2bf((float)images[g.src + (int64_t)y * g.src_pitch + x] / 255.f);
}

// Forward 3x3 conv + bias + relu for a 16-cell x 4-row tile (one wave per row).
template <bool FIRST>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint8_t* __restrict__ images, const short* __restrict__ X,
                                                  const float* __restrict__ Wl, const float* __restrict__ bl,
                                                  short* __restrict__ Y, const CnnImage* __restrict__ imgs, int nimg) {
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const CnnImage& g = imgs[find_cnn_image(imgs, nimg, tile)];
    const int lt = tile - g.tile0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cy = (lt / g.tiles_x) * kCnnTileH + wave;
    const int px = (lt % g.tiles_x) * kCnnTileW + (lane & 15);
    const int kb = lane >> 4, half = kb >> 1, c8 = (kb & 1) * 8;
    if (cy >= g.H4) return;
    s8 a[kTapPairs];
#pragma unroll
    for (int m = 0; m < kTapPairs; ++m) {
        const int t = 2 * m + half;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[m][j] = t < 9 ? f2bf(Wl[(t * CC + c8 + j) * CC + (lane & 15)]) : (short)0;
    }
    f4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = bl[4 * kb + r];
#pragma unroll
    for (int m = 0; m < kTapPairs; ++m) {
        const int t = 2 * m + half;
        const int yy = cy + t / 3 - 1, xx = px + t % 3 - 1;
        s8 b = {0, 0, 0, 0, 0, 0, 0, 0};
        if (t < 9 && yy >= 0 && yy < g.H4 && xx >= 0 && xx < g.W4) {
            if constexpr (FIRST) {
                const s4 lo = s2d_frag(images, g, yy, xx, 2 * (kb & 1)), hi = s2d_frag(images, g, yy, xx, 2 * (kb & 1) + 1);
                b = s8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            } else {
                b = *reinterpret_cast<const s8*>(X + (g.cell0 + (int64_t)yy * g.W4 + xx) * CC + c8);
            }
        }
        acc = mfma32(a[m], b, acc);
    }
    if (px < g.W4) {
        s4 o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = f2bf(fmaxf(acc[r], 0.f));
        *reinterpret_cast<s4*>(Y + (g.cell0 + (int64_t)cy * g.W4 + px) * CC + 4 * kb) = o;
    }
}

// 1x1 head: logits and/or mask bits, one thread per cell.
__global__ __launch_bounds__(256) void k_head(const short* __restrict__ X4, const float* __restrict__ P,
                                              const CnnImage* __restrict__ imgs, int nimg, int64_t ncells,
                                              float* __restrict__ logits, uint8_t* __restrict__ mask, float zthr) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const float* Wh = P + kCnnLayers * LAYER_P;
    const float* bh = Wh + CC * NHD;
    float x[CC];
    const uint4* src = reinterpret_cast<const uint4*>(X4 + c * CC);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const uint4 v = src[q];
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            x[8 * q + 2 * h] = __uint_as_float(w4[h] << 16);
            x[8 * q + 2 * h + 1] = __uint_as_float(w4[h] & 0xFFFF0000u);
        }
    }
    float z[NHD];
#pragma unroll
    for (int o = 0; o < NHD; ++o) {
        float s = bh[o];
#pragma unroll
        for (int ch = 0; ch < CC; ++ch) s = fmaf(x[ch], Wh[ch * NHD + o], s);
        z[o] = s;
    }
    if (logits) {
#pragma unroll
        for (int o = 0; o < NHD; ++o) logits[c * NHD + o] = z[o];
    }
    if (mask) {
        const int n_oct = imgs[find_cell_image(imgs, nimg, c)].n_oct;
        uint32_t bits = 0;
#pragma unroll
        for (int o = 0; o < NHD; ++o)
            if (o < n_oct && z[o] > zthr) bits |= 1u << o;
        mask[c] = (uint8_t)bits;
    }
}

// Fused inference: the four convolutions and the head for a 32 x 16 block of
// output cells in one workgroup, with every activation kept in LDS (no
// activation goes to HBM).  The workgroup stages the s2d input over the block
// plus a 4-cell halo (one cell per layer) and each layer writes its output
// over a region one cell smaller on every side, so the last layer covers
// exactly the block.  Cells outside the image are written as zeros at every
// layer, which is the zero padding of each convolution.  The arithmetic is
// the unfused kernels' (same fragments, same MFMA order, same bf16
// roundings), so logits and mask bits are identical to theirs.
constexpr int FTW = kCnnFusedW, FTH = kCnnFusedH, FHALO = kCnnLayers;
constexpr int FFW = FTW + 2 * FHALO, FFH = FTH + 2 * FHALO;   // 40 x 24 frame
constexpr int FSTR = CC;                                       // shorts per cell (32 B, 16-byte aligned reads)


// MFMA weight fragments of all layers, packed once per forward call:
// frag[((l * kTapPairs + m) * 64 + lane) * 8 + j] is exactly the A operand
// element j that lane `lane` of k_conv_fwd builds for tap pair m of layer l.
__global__ void k_cnn_pack(const float* __restrict__ P, short* __restrict__ frag) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kCnnLayers * kTapPairs * 64; i += gridDim.x * blockDim.x) {
        const int lane = i % 64, m = (i / 64) % kTapPairs, l = i / (64 * kTapPairs);
        const int kb = lane >> 4, t = 2 * m + (kb >> 1), c8 = (kb & 1) * 8;
        const float* Wl = P + l * LAYER_P;
#pragma unroll
        for (int j = 0; j < 8; ++j) frag[i * 8 + j] = t < 9 ? f2bf(Wl[(t * CC + c8 + j) * CC + (lane & 15)]) : (short)0;
    }
}

constexpr int FTHREADS = 512;                       // 8 waves: twice the latency hiding of 4 at the same LDS
constexpr int FSTAGE = (FFH * FFW * 4 + FTHREADS - 1) / FTHREADS;   // 4-pixel cell rows staged per lane

__global__ __launch_bounds__(FTHREADS, 2) void k_cnn_infer(const uint8_t* __restrict__ images, const float* __restrict__ P,
                                                      const short* __restrict__ frag,
                                                      const CnnImage* __restrict__ imgs,
                                                      const int32_t* __restrict__ owner,
                                                      float* __restrict__ logits, uint8_t* __restrict__ mask,
                                                      float zthr) {
    __shared__ __align__(16) short buf[2][FFH * FFW * FSTR];
    __shared__ short lut[256];
    __shared__ float head[CC * NHD + NHD];
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const CnnImage& g = imgs[owner[tile]];   // per-tile owner table: one load, no search
    const int lt = tile - g.ftile0;
    const int ty0 = (lt / g.ftiles_x) * FTH, tx0 = (lt % g.ftiles_x) * FTW;
    const int oy = ty0 - FHALO, ox = tx0 - FHALO;   // image cell of frame (0, 0)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kb = lane >> 4;
    const int H4 = g.H4, W4 = g.W4;   // read once (the layer loops test every cell against them)

    // u8 -> bf16(u / 255) table (the same expression as s2d_frag)
    if (threadIdx.x < 256) lut[threadIdx.x] = f2bf((float)threadIdx.x / 255.f);
    for (int i = threadIdx.x; i < CC * NHD + NHD; i += blockDim.x) head[i] = P[kCnnLayers * LAYER_P + i];
    // layer 0 input: s2d of the frame, zero outside the image.  Lanes take
    // consecutive cells of one pixel row (contiguous 4-byte groups); all
    // loads are issued before the first conversion.
    uint32_t px[FSTAGE];
#pragma unroll
    for (int k = 0; k < FSTAGE; ++k) {
        const int it = threadIdx.x + k * FTHREADS;
        const int fx = it % FFW, r4 = (it / FFW) & 3, fy = it / (FFW * 4);
        const int cy = oy + fy, cx = ox + fx;
        px[k] = 0;
        if (it < FFH * FFW * 4 && cy >= 0 && cy < H4 && cx >= 0 && cx < W4) {
            const int y = min(4 * cy + r4, g.H - 1);
            const uint8_t* row = images + g.src + (int64_t)y * g.src_pitch;
            const int x0 = 4 * cx;
            if (x0 + 3 < g.W && ((uintptr_t)(row + x0) & 3) == 0) {
                px[k] = *reinterpret_cast<const uint32_t*>(row + x0);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) px[k] |= (uint32_t)row[min(x0 + j, g.W - 1)] << (8 * j);
            }
        }
    }
    __syncthreads();   // lut
#pragma unroll
    for (int k = 0; k < FSTAGE; ++k) {
        const int it = threadIdx.x + k * FTHREADS;
        if (it >= FFH * FFW * 4) break;
        const int fx = it % FFW, r4 = (it / FFW) & 3, fy = it / (FFW * 4);
        const int cy = oy + fy, cx = ox + fx;
        s4 v = {0, 0, 0, 0};
        if (cy >= 0 && cy < H4 && cx >= 0 && cx < W4) {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = lut[(px[k] >> (8 * j)) & 255u];
        }
        *reinterpret_cast<s4*>(&buf[0][(fy * FFW + fx) * FSTR + 4 * r4]) = v;
    }
    const int half = kb >> 1, c8 = (kb & 1) * 8;
    s8 a[kTapPairs];
    const s8* fr = reinterpret_cast<const s8*>(frag);
#pragma unroll
    for (int m = 0; m < kTapPairs; ++m) a[m] = fr[m * 64 + lane];
    __syncthreads();

    // The layers are unrolled, so each layer's output region is a constant
    // and a cell index splits into (row, column) by constant division.  A
    // lane's B operand of tap pair m is read at a per-lane base plus a
    // constant offset: the base points at tap 0 of its cell (the cell at
    // (-1, -1)), shifted for the lanes carrying the pair's second tap by
    // that tap's distance from the first, which is one cell for pairs 0, 2
    // and 3 and FFW - 2 cells for pair 1; pair 4's second tap is zero.  All
    // ten loads of a step are issued before its MFMAs.
    const int c8b = 2 * c8;                 // byte offset of this lane's 8 channels
#pragma unroll
    for (int l = 0; l < kCnnLayers; ++l) {
        f4 bias;
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[r] = P[l * LAYER_P + CONV_W + 4 * kb + r];
        // the next layer's fragments load while this layer computes
        s8 an[kTapPairs];
        const int ln = l + 1 < kCnnLayers ? l + 1 : l;
#pragma unroll
        for (int m = 0; m < kTapPairs; ++m) an[m] = fr[(ln * kTapPairs + m) * 64 + lane];
        const char* X = reinterpret_cast<const char*>(buf[l & 1]);
        short* Y = buf[(l + 1) & 1];
        const int lo = l + 1, C = FFW - 2 * lo, n = (FFH - 2 * lo) * C;
        constexpr int CB = FSTR * 2;        // bytes per cell
        // tap t = 3 (dy + 1) + (dx + 1) at byte offset (dy + 1) FFW CB + (dx + 1) CB from tap 0
        auto toff = [](int t) { return ((t / 3) * FFW + t % 3) * CB; };
        for (int q0 = wave * 32; q0 < n; q0 += 32 * (FTHREADS / 64)) {
            int fy[2], fx[2];
            const char* pa[2];
            const char* pb[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = min(q0 + 16 * h + (lane & 15), n - 1);
                fy[h] = lo + q / C;
                fx[h] = lo + q % C;
                const char* base = X + ((fy[h] - 1) * FFW + fx[h] - 1) * CB + c8b;
                pa[h] = base + half * CB;
                pb[h] = base + half * (FFW - 2) * CB;
            }
            s8 b[kTapPairs][2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                b[0][h] = *reinterpret_cast<const s8*>(pa[h] + toff(0));
                b[1][h] = *reinterpret_cast<const s8*>(pb[h] + toff(2));
                b[2][h] = *reinterpret_cast<const s8*>(pa[h] + toff(4));
                b[3][h] = *reinterpret_cast<const s8*>(pa[h] + toff(6));
                b[4][h] = *reinterpret_cast<const s8*>(pa[h] - half * CB + toff(8));
            }
            f4 acc[2] = {bias, bias};
#pragma unroll
            for (int m = 0; m < kTapPairs; ++m)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // (the tenth tap's lanes read tap 8's cell again: its A
                    // fragment is zero and every activation is finite and
                    // non-negative, so those products add exact zeros)
                    acc[h] = mfma32(a[m], b[m][h], acc[h]);
                }
            // relu, bf16, zero outside the image: computed for every lane and
            // selected (no branch per element), one 8-byte store per cell
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cy = oy + fy[h], cx = ox + fx[h];
                const bool in = (unsigned)cy < (unsigned)H4 && (unsigned)cx < (unsigned)W4;
                uint2 o;
                o.x = f2bf2(relu(acc[h][0]), relu(acc[h][1]));
                o.y = f2bf2(relu(acc[h][2]), relu(acc[h][3]));
                o.x = in ? o.x : 0u;
                o.y = in ? o.y : 0u;
                if (q0 + 16 * h + (lane & 15) < n)
                    *reinterpret_cast<uint2*>(&Y[(fy[h] * FFW + fx[h]) * FSTR + 4 * kb]) = o;
            }
        }
#pragma unroll
        for (int m = 0; m < kTapPairs; ++m) a[m] = an[m];
        __syncthreads();
    }

    // head on the last layer's output (kCnnLayers is even: it is in buf[0])
    const short* X4 = buf[kCnnLayers & 1];
    for (int q = threadIdx.x; q < FTH * FTW; q += blockDim.x) {
        const int cy = ty0 + q / FTW, cx = tx0 + q % FTW;
        if (cy >= H4 || cx >= W4) continue;
        const short* xs = &X4[((FHALO + q / FTW) * FFW + FHALO + q % FTW) * FSTR];
        float x[CC];
#pragma unroll
        for (int ch = 0; ch < CC; ++ch) x[ch] = bf2f(xs[ch]);
        const int64_t c = g.cell0 + (int64_t)cy * W4 + cx;
        uint32_t bits = 0;
#pragma unroll
        for (int o = 0; o < NHD; ++o) {
            float s = head[CC * NHD + o];
#pragma unroll
            for (int ch = 0; ch < CC; ++ch) s = fmaf(x[ch], head[ch * NHD + o], s);
            if (logits) logits[c * NHD + o] = s;
            if (o < g.n_oct && s > zthr) bits |= 1u << o;
        }
        if (mask) mask[c] = (uint8_t)bits;
    }
}

__device__ __forceinline__ float softplus(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }

// Head backward + loss: per cell dZ, the masked gradient dP4 = (dZ Wh^T) *
// (X4 > 0) as bf16, and grid-stride partial sums of dWh, dbh and the loss
// reduced per wave and added to the global gradient with atomics.  The loss
// is the mean over images of each image's mean over cells and its octaves.
__global__ __launch_bounds__(256) void k_head_bwd(const short* __restrict__ X4, const float* __restrict__ P,
                                                  const float* __restrict__ logits, const uint32_t* __restrict__ labels,
                                                  const float* __restrict__ pos_w, const CnnImage* __restrict__ imgs,
                                                  int nimg, int64_t ncells, short* __restrict__ dP4,
                                                  float* __restrict__ grad, float* __restrict__ loss) {
    const float* Wh = P + kCnnLayers * LAYER_P;
    float gW[CC * NHD], gb[NHD], lsum = 0.f;
#pragma unroll
    for (int i = 0; i < CC * NHD; ++i) gW[i] = 0.f;
#pragma unroll
    for (int o = 0; o < NHD; ++o) gb[o] = 0.f;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * blockDim.x) {
        const CnnImage& g = imgs[find_cell_image(imgs, nimg, c)];
        const float scale = 1.f / ((float)g.H4 * (float)g.W4 * (float)g.n_oct * (float)nimg);
        const uint32_t y = labels[c];
        float x[CC];
#pragma unroll
        for (int ch = 0; ch < CC; ++ch) x[ch] = bf2f(X4[c * CC + ch]);
        float dz[NHD];
#pragma unroll
        for (int o = 0; o < NHD; ++o) {
            dz[o] = 0.f;
            if (o < g.n_oct) {
                const float z = logits[c * NHD + o];
                const float yo = (float)((y >> o) & 1u), w = pos_w[o];
                const float s = 1.f / (1.f + expf(-z));
                dz[o] = (s * (w * yo + 1.f - yo) - w * yo) * scale;
                lsum += (w * yo * softplus(-z) + (1.f - yo) * softplus(z)) * scale;
            }
            gb[o] += dz[o];
        }
        short out[CC];
#pragma unroll
        for (int ch = 0; ch < CC; ++ch) {
            float d = 0.f;
#pragma unroll
            for (int o = 0; o < NHD; ++o) {
                d = fmaf(Wh[ch * NHD + o], dz[o], d);
                gW[ch * NHD + o] = fmaf(x[ch], dz[o], gW[ch * NHD + o]);
            }
            out[ch] = f2bf(x[ch] > 0.f ? d : 0.f);
        }
        s4* dst = reinterpret_cast<s4*>(dP4 + c * CC);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = s4{out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]};
    }
    const int lane = threadIdx.x & 63;
    float* gWh = grad + kCnnLayers * LAYER_P;
    float* gbh = gWh + CC * NHD;
#pragma unroll
    for (int i = 0; i < CC * NHD; ++i) {
        float v = gW[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) atomicAdd(&gWh[i], v);
    }
#pragma unroll
    for (int o = 0; o < NHD; ++o) {
        float v = gb[o];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) atomicAdd(&gbh[o], v);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) atomicAdd(loss, lsum);
}

// Input gradient of layer l: dX_{l-1}[p][ci] = sum_t sum_co W[t][ci][co]
// dP_l[p - d_t][co], then times (X_{l-1} > 0) to give dP_{l-1} (bf16).
__global__ __launch_bounds__(256) void k_conv_bwd_data(const short* __restrict__ dP, const float* __restrict__ Wl,
                                                       const short* __restrict__ Xprev, short* __restrict__ dPprev,
                                                       const CnnImage* __restrict__ imgs, int nimg) {
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const CnnImage& g = imgs[find_cnn_image(imgs, nimg, tile)];
    const int lt = tile - g.tile0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cy = (lt / g.tiles_x) * kCnnTileH + wave;
    const int px = (lt % g.tiles_x) * kCnnTileW + (lane & 15);
    const int kb = lane >> 4;
    if (cy >= g.H4) return;
    s4 a[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) a[t][j] = f2bf(Wl[(t * CC + (lane & 15)) * CC + 4 * kb + j]);
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = cy - (t / 3 - 1), xx = px - (t % 3 - 1);
        s4 b = {0, 0, 0, 0};
        if (yy >= 0 && yy < g.H4 && xx >= 0 && xx < g.W4)
            b = *reinterpret_cast<const s4*>(dP + (g.cell0 + (int64_t)yy * g.W4 + xx) * CC + 4 * kb);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t], b, acc, 0, 0, 0);
    }
    if (px < g.W4) {
        const int64_t off = (g.cell0 + (int64_t)cy * g.W4 + px) * CC + 4 * kb;
        const s4 xp = *reinterpret_cast<const s4*>(Xprev + off);
        s4 o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = f2bf(bf2f(xp[r]) > 0.f ? acc[r] : 0.f);
        *reinterpret_cast<s4*>(dPprev + off) = o;
    }
}

// Weight and bias gradients of layer l: dW[t][ci][co] = sum_p X_{l-1}[p + d_t][ci]
// dP_l[p][co] as MFMAs with K = 16 pixels of one row; grid-stride over
// 16-cell row chunks, per-lane partial sums added with global atomics.
template <bool FIRST>
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const uint8_t* __restrict__ images,
                                                         const short* __restrict__ Xprev, const short* __restrict__ dP,
                                                         const CnnImage* __restrict__ imgs, int nimg, int nchunks,
                                                         float* __restrict__ gW, float* __restrict__ gb) {
    const int lane = threadIdx.x & 63, kb = lane >> 4, li = lane & 15;
    const int wave_g = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    f4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (int ch = wave_g; ch < nchunks; ch += nwaves) {
        // chunk -> (image, row, 16-cell segment): chunks of an image are
        // numbered row-major with tiles_x segments per row
        int lo = 0, hi = nimg - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (imgs[mid].chunk0 <= ch) lo = mid;
            else hi = mid - 1;
        }
        const CnnImage& g = imgs[lo];
        const int lc = ch - g.chunk0;
        const int cy = lc / g.tiles_x, cx0 = (lc % g.tiles_x) * kCnnTileW;
        s4 b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xx = cx0 + 4 * kb + j;
            b[j] = xx < g.W4 ? dP[(g.cell0 + (int64_t)cy * g.W4 + xx) * CC + li] : (short)0;
            bsum += bf2f(b[j]);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = cy + t / 3 - 1;
            s4 a;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xx = cx0 + 4 * kb + j + t % 3 - 1;
                short v = 0;
                if (yy >= 0 && yy < g.H4 && xx >= 0 && xx < g.W4) {
                    if constexpr (FIRST) v = s2d_chan(images, g, yy, xx, li);
                    else v = Xprev[(g.cell0 + (int64_t)yy * g.W4 + xx) * CC + li];
                }
                a[j] = v;
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
    // acc[t][r] = dW[t][ci = 4 kb + r][co = li]
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) atomicAdd(&gW[(t * CC + 4 * kb + r) * CC + li], acc[t][r]);
    bsum += __shfl_xor(bsum, 16);
    bsum += __shfl_xor(bsum, 32);
    if (lane < 16) atomicAdd(&gb[li], bsum);
}

__global__ void k_fill(float* p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Adam (Kingma and Ba 2015) with bias correction on fp32 master weights.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Cell labels from detector keypoints: bit o of the cell holding
// (ix 2^o, iy 2^o) / 4 for every keypoint of octave o.
__global__ void k_labels(const cdvs_keypoint* __restrict__ kp, const int32_t* __restrict__ count, int kp_cap,
                         const CnnImage* __restrict__ imgs, int nimg, uint32_t* __restrict__ labels) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int img = (int)(s / kp_cap), i = (int)(s % kp_cap);
    if (img >= nimg || i >= count[img]) return;
    const cdvs_keypoint k = kp[s];
    if (k.octave < 0 || k.octave >= kMaxOctaves) return;
    const CnnImage& g = imgs[img];
    const int cx = min((k.ix << k.octave) >> 2, g.W4 - 1), cy = min((k.iy << k.octave) >> 2, g.H4 - 1);
    atomicOr(&labels[g.cell0 + (int64_t)cy * g.W4 + cx], 1u << k.octave);
}

// Active-cell count per (image, octave) of a mask, for the dense fallback.
// Active cells per (image, octave) of a mask, one 1024-lane workgroup per
// image: the image's cell bytes are read 16 at a time from the first
// 16-byte boundary (the bytes before it and after the last whole group one
// at a time), and octave o's count of a 4-byte word is the population count
// of bit o of its four bytes.
constexpr int kCountThreads = 1024;

__device__ __forceinline__ void count_word(uint32_t x, int (&loc)[NHD]) {
#pragma unroll
    for (int o = 0; o < NHD; ++o) loc[o] += __popc(x & (0x01010101u << o));
}

__global__ __launch_bounds__(kCountThreads) void k_mask_count(const uint8_t* __restrict__ mask,
                                                             const CnnImage* __restrict__ imgs,
                                                             int32_t* __restrict__ active) {
    __shared__ int cnt[NHD];
    const CnnImage& g = imgs[blockIdx.x];
    if (threadIdx.x < NHD) cnt[threadIdx.x] = 0;
    __syncthreads();
    int loc[NHD] = {0, 0, 0, 0, 0, 0};
    const int64_t n = (int64_t)g.H4 * g.W4;
    const uint8_t* m = mask + g.cell0;
    const int64_t head = min(n, (int64_t)((16u - ((uint32_t)(uintptr_t)m & 15u)) & 15u));
    const int64_t ng = (n - head) / 16;   // whole 16-byte groups
    const uint4* q = reinterpret_cast<const uint4*>(m + head);
    for (int64_t c = threadIdx.x; c < ng; c += blockDim.x) {
        const uint4 v = q[c];
        count_word(v.x, loc);
        count_word(v.y, loc);
        count_word(v.z, loc);
        count_word(v.w, loc);
    }
    // the bytes before the first group and after the last
    const int64_t tail0 = head + 16 * ng, rest = head + (n - tail0);
    for (int64_t j = threadIdx.x; j < rest; j += blockDim.x) count_word(m[j < head ? j : tail0 + (j - head)], loc);
#pragma unroll
    for (int o = 0; o < NHD; ++o)
        if (loc[o]) atomicAdd(&cnt[o], loc[o]);
    __syncthreads();
    if (threadIdx.x < kMaxOctaves) active[blockIdx.x * kMaxOctaves + threadIdx.x] = threadIdx.x < NHD ? cnt[threadIdx.x] : 0;
}

}  // namespace

hipError_t launch_cnn_infer(const uint8_t* images, const float* params, short* frag, const CnnImage* imgs,
                            const int32_t* owner, int ntiles, float* logits, uint8_t* mask, float zthr, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cnn_pack, dim3(9), dim3(256), 0, s, params, frag);
    hipLaunchKernelGGL(k_cnn_infer, dim3(ntiles), dim3(FTHREADS), 0, s, images, params, frag, imgs, owner, logits,
                       mask, zthr);
    return hipGetLastError();
}

hipError_t launch_cnn_forward(const uint8_t* images, const float* params, short* acts, int64_t ncells,
                              const CnnImage* imgs, int nimg, int ntiles, float* logits, uint8_t* mask, float zthr,
                              hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    for (int l = 0; l < kCnnLayers; ++l) {
        const float* W = params + l * LAYER_P;
        const float* b = W + CONV_W;
        short* Y = acts + (int64_t)l * ncells * CC;
        if (l == 0)
            hipLaunchKernelGGL(k_conv_fwd<true>, dim3(ntiles), dim3(256), 0, s, images, nullptr, W, b, Y, imgs, nimg);
        else
            hipLaunchKernelGGL(k_conv_fwd<false>, dim3(ntiles), dim3(256), 0, s, images,
                               acts + (int64_t)(l - 1) * ncells * CC, W, b, Y, imgs, nimg);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int blocks = (int)((ncells + 255) / 256);
    hipLaunchKernelGGL(k_head, dim3(blocks), dim3(256), 0, s, acts + (int64_t)(kCnnLayers - 1) * ncells * CC, params,
                       imgs, nimg, ncells, logits, mask, zthr);
    return hipGetLastError();
}

hipError_t launch_cnn_backward(const uint8_t* images, const float* params, const short* acts, int64_t ncells,
                               const CnnImage* imgs, int nimg, int ntiles, int nchunks, const float* logits,
                               const uint32_t* labels, const float* pos_w, short* dbuf, float* grad, float* loss,
                               int wgrid, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, grad, kCnnParams, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, loss, 1, 0.f);
    short* dA = dbuf;
    short* dB = dbuf + ncells * CC;
    const int hgrid = std::max(1, std::min((int)((ncells + 255) / 256), wgrid));
    hipLaunchKernelGGL(k_head_bwd, dim3(hgrid), dim3(256), 0, s, acts + (int64_t)(kCnnLayers - 1) * ncells * CC,
                       params, logits, labels, pos_w, imgs, nimg, ncells, dA, grad, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = kCnnLayers - 1; l >= 0; --l) {
        const float* W = params + l * LAYER_P;
        float* gW = grad + l * LAYER_P;
        float* gb = gW + CONV_W;
        const short* Xprev = l > 0 ? acts + (int64_t)(l - 1) * ncells * CC : nullptr;
        if (l == 0)
            hipLaunchKernelGGL(k_conv_bwd_weight<true>, dim3(wgrid), dim3(256), 0, s, images, nullptr, dA, imgs, nimg,
                               nchunks, gW, gb);
        else
            hipLaunchKernelGGL(k_conv_bwd_weight<false>, dim3(wgrid), dim3(256), 0, s, images, Xprev, dA, imgs, nimg,
                               nchunks, gW, gb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (l > 0) {
            hipLaunchKernelGGL(k_conv_bwd_data, dim3(ntiles), dim3(256), 0, s, dA, W, Xprev, dB, imgs, nimg);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            short* t = dA;
            dA = dB;
            dB = t;
        }
    }
    return hipSuccess;
}

hipError_t launch_cnn_adam(float* p, const float* g, float* m, float* v, int step, float lr, float b1, float b2,
                           float eps, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, p, g, m, v, kCnnParams, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_cnn_labels(const cdvs_keypoint* kp, const int32_t* count, int kp_cap, const CnnImage* imgs, int nimg,
                             int64_t ncells, uint32_t* labels, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0, s, labels, ncells);
    const int64_t slots = (int64_t)nimg * kp_cap;
    hipLaunchKernelGGL(k_labels, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, s, kp, count, kp_cap, imgs, nimg,
                       labels);
    return hipGetLastError();
}

hipError_t launch_mask_count(const uint8_t* mask, const CnnImage* imgs, int nimg, int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_count, dim3(nimg), dim3(kCountThreads), 0, s, mask, imgs, active);
    return hipGetLastError();
}

}  // namespace cdvs
