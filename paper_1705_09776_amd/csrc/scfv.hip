// SCFV global aggregation on gfx950 (Sec. III-D, Eqs. (6)-(8); Sec. IV-C,
// Eqs. (9)-(14)): per image, every local descriptor d_t (128-D) is projected
// by PCA to x_t = A (d_t - m) (32-D), scored against a diagonal GMM of 512
// components, and the posterior-weighted gradients with respect to the
// components' means and variances are accumulated; each component's mean
// gradient gives delta (the spread of its 32 entries), by which the
// components are ranked, and one sign bit per gradient entry.
//
// The paper turns these per-descriptor formulas into matrix products (its
// Eqs. (10), (12), (14)); here they are three MFMA contractions per tile of
// 32 descriptors, all in one workgroup per image:
//   X   = (D - m) A^T                              16x16x4 f32 MFMA (4 waves)
//   L   = [X | X.*X] [M./V ; -1/(2V)]^T + c        32x32x2 f32 MFMA, K = 64
//         (c_j = log w_j - sum log V_j / 2 - sum M_j.^2 ./ V_j / 2), the
//         log of w_j p_j(x_t) up to a constant; a softmax over the 512
//         components gives the posteriors Q (Eq. (6))
//   S  += Q^T [X | X.*X]                            32x32x2 f32 MFMA, K = 32
// and the epilogue forms GM = (S1 - S0 M) ./ sigma and GV = (S2 - 2 S1 .* M
// + S0 (M.*M - V)) ./ V (Eqs. (12), (14)), scaled as Eq. (7) by
// 1/(K sqrt(w)) (and 1/(K sqrt(2w)) for the variances).  FP32 operands and
// accumulation throughout (the posteriors are exponentials of sums near
// 100 in magnitude: bf16 operands would not resolve them).
//
// MFMA layouts (wave64): 32x32x2 f32: lane l holds A[l%32][l/32] and
// B[l/32][l%32], and D[8(i/4) + 4(l/32) + i%4][l%32] in register i = 0..15;
// 16x16x4 f32: A[l%16][l/16], B[l/16][l%16], D[4(l/16) + r][l%16], r = 0..3.
#include <algorithm>
#include <mutex>

#include "cdvs_internal.h"

namespace cdvs {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int NC = kScfvComponents;   // 512
constexpr int PD = kScfvDim;          // 32
constexpr int TD = 32;                // descriptors per tile
constexpr int NW = 8;                 // waves per workgroup
constexpr int CPW = NC / NW;          // components per wave: 64 (two 32-wide tiles)
constexpr int DSTR = 132;             // LDS row stride of the descriptor tile (conflict-free A reads)
constexpr int XRS = 72;               // LDS row stride of [X | X.*X] by rows (halves on disjoint banks)
static_assert(NC == NW * CPW && CPW == 64 && PD == 32, "tiling assumes 512 components of 32 dimensions");

__device__ __forceinline__ f16v mfma32(float a, float b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Per-component constants of one call, derived on the device from the
// caller's model: B[j][0..31] = M_j ./ V_j, B[j][32..63] = -1 / (2 V_j);
// c_j; 1/sqrt(w_j); 1/sigma_jk.
__global__ __launch_bounds__(256) void k_scfv_prep(const float* __restrict__ w, const float* __restrict__ means,
                                                   const float* __restrict__ vars, float* __restrict__ prep) {
    const int j = blockIdx.x * 8 + (threadIdx.x >> 5), k = threadIdx.x & 31;
    if (j >= NC) return;
    const float m = means[j * PD + k], v = vars[j * PD + k];
    float* B = prep + kScfvPrepB;
    B[j * 64 + k] = m / v;
    B[j * 64 + 32 + k] = -0.5f / v;
    prep[kScfvPrepIsig + j * PD + k] = 1.f / sqrtf(v);
    float t = logf(v) + m * m / v;   // summed over the 32 lanes of this component
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (k == 0) {
        prep[kScfvPrepC + j] = logf(w[j]) - 0.5f * t;
        prep[kScfvPrepRsw + j] = 1.f / sqrtf(w[j]);
    }
}

// Reductions over each 32-lane half of the wave, the result in every lane:
// within each 16-lane row by DPP (quad permutes [1,0,3,2] and [2,3,0,1],
// then the half-row and row mirrors, each combining a lane group with the
// other half of the next larger group), then across the half's two rows by
// one swizzle (lane ^ 16 within 32-lane groups).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float xor16(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}
__device__ __forceinline__ float half_max(float v) {
    v = fmaxf(v, dpp<0xB1>(v));
    v = fmaxf(v, dpp<0x4E>(v));
    v = fmaxf(v, dpp<0x141>(v));
    v = fmaxf(v, dpp<0x140>(v));
    return fmaxf(v, xor16(v));
}
__device__ __forceinline__ float half_sum(float v) {
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    return v + xor16(v);
}

// Output stage of one image, shared by the one-workgroup-per-image kernel
// and the kernel that completes split images: s0s[] holds S0 of every
// component, acc1/acc2 this lane's S1/S2 entries in the 32x32 MFMA
// accumulator layout (component 64 wave + 32 t + 8 (i/4) + 4 (lane/32) +
// i%4, dimension lane%32).  Writes the gradients (Eqs. (7), (12), (14)),
// delta (Eq. (8)), the sign bits and the component order.
__device__ __forceinline__ void scfv_output(int img, int K, int wave, int lane, const float* s0s,
                                            const f16v (&acc1)[2], const f16v (&acc2)[2],
                                            const float* __restrict__ means, const float* __restrict__ vars,
                                            const float* __restrict__ prep, float* __restrict__ gm_out,
                                            float* __restrict__ gv_out, float* __restrict__ delta_out,
                                            int32_t* __restrict__ order_out, uint32_t* __restrict__ bits_out,
                                            float* skey, int* sidx) {
    const int tid = threadIdx.x, h = lane >> 5, k = lane & 31;
    const float invK = K > 0 ? 1.f / (float)K : 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int comp = CPW * wave + 32 * t + 8 * (i >> 2) + 4 * h + (i & 3);
            const float S0 = s0s[comp], S1 = acc1[t][i], S2 = acc2[t][i];
            const float m = means[comp * PD + k], v = vars[comp * PD + k];
            const float isg = prep[kScfvPrepIsig + comp * PD + k], rsw = prep[kScfvPrepRsw + comp];
            const float gm = (S1 - S0 * m) * isg * (invK * rsw);
            const float gv = (S2 - 2.f * S1 * m + S0 * (m * m - v)) * (isg * isg) * (invK * rsw * 0.70710678118654752f);
            const int64_t o = ((int64_t)img * NC + comp) * PD + k;
            gm_out[o] = gm;
            gv_out[o] = gv;
            const float mean = half_sum(gm) * (1.f / PD);
            const float dv = gm - mean;
            const float dl = sqrtf(half_sum(dv * dv) * (1.f / PD));
            const uint64_t bm = __ballot(gm > 0.f), bv = __ballot(gv > 0.f);
            if (k == 0) {
                delta_out[(int64_t)img * NC + comp] = dl;
                bits_out[((int64_t)img * NC + comp) * 2] = (uint32_t)(bm >> (32 * h));
                bits_out[((int64_t)img * NC + comp) * 2 + 1] = (uint32_t)(bv >> (32 * h));
                skey[comp] = dl;
                sidx[comp] = comp;
            }
        }
    __syncthreads();
    // rank by delta, descending, ties by lower index: bitonic sort of 512
    // (key, index) pairs, one per thread
    for (int size = 2; size <= NC; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int j = tid ^ stride;
            if (j > tid) {
                const float ka = skey[tid], kb = skey[j];
                const int ia = sidx[tid], ib = sidx[j];
                // a before b: larger key, or equal key and lower index
                const bool a_first = ka > kb || (ka == kb && ia < ib);
                const bool up = (tid & size) == 0;
                if (up != a_first) {
                    skey[tid] = kb;
                    skey[j] = ka;
                    sidx[tid] = ib;
                    sidx[j] = ia;
                }
            }
            __syncthreads();
        }
    order_out[(int64_t)img * NC + tid] = sidx[tid];
}

// One workgroup of 8 waves per image (SPLIT = false), or per part of an
// image (SPLIT = true: image blockIdx.x / splits takes descriptor tiles
// [part * tiles_per_part, (part + 1) * tiles_per_part) and writes its sums
// S0, S1, S2 to partial block blockIdx.x, which k_scfv_join adds up).
// Wave w owns components [64 w, 64 w + 64): their logits and their
// gradient accumulators live in its registers for the whole range.
template <bool SPLIT>
__global__ __launch_bounds__(512) void k_scfv(const float* __restrict__ desc, const int32_t* __restrict__ count,
                                              int kp_cap, int splits, int tiles_per_part,
                                              const float* __restrict__ pca_mean,
                                              const float* __restrict__ pca_matrix, const float* __restrict__ means,
                                              const float* __restrict__ vars, const float* __restrict__ prep,
                                              float* __restrict__ partial, float* __restrict__ gm_out,
                                              float* __restrict__ gv_out, float* __restrict__ delta_out,
                                              int32_t* __restrict__ order_out, uint32_t* __restrict__ bits_out) {
    __shared__ float Dl[TD * DSTR];        // descriptor tile minus the PCA mean
    __shared__ float XXt[64 * TD];         // [X | X.*X] by columns: [k][descriptor]
    __shared__ float XXr[TD * XRS];        // [X | X.*X] by rows: [descriptor][k]
    __shared__ float redm[NW][TD], reds[NW][TD];
    __shared__ float rowq[TD][2];          // per descriptor: global max, 1/sum (0 for padding rows)
    __shared__ float s0s[NC];
    __shared__ float skey[NC];
    __shared__ int sidx[NC];

    const int img = SPLIT ? blockIdx.x / splits : blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, h = lane >> 5, c32 = lane & 31;
    const int K = min(max(count[img], 0), kp_cap);
    // descriptor range of this workgroup: [tbeg, tend)
    const int tbeg = SPLIT ? min(K, (blockIdx.x % splits) * tiles_per_part * TD) : 0;
    const int tend = SPLIT ? min(K, tbeg + tiles_per_part * TD) : K;
    const float* D = desc + (int64_t)img * kp_cap * kDescDim;
    const float* Bp = prep + kScfvPrepB;

    // logits B operand of this wave: B[comp 64w + 32t + l%32][k = 2s + l/32]
    float bf[2][32];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < 32; ++s) bf[t][s] = Bp[(CPW * wave + 32 * t + c32) * 64 + 2 * s + h];
    float cc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) cc[t] = prep[kScfvPrepC + CPW * wave + 32 * t + c32];

    f16v acc1[2], acc2[2];   // [t]: S1 (columns x) and S2 (columns x^2) of this wave's comps
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        acc1[t] = f16v{};
        acc2[t] = f16v{};
    }
    float s0[2] = {0.f, 0.f};

    // The descriptor tile is staged through registers: each thread holds
    // two float4s (the same column group q of rows r and r + 16) and loads
    // the next tile's while the current one is computed, so the global
    // load's latency is hidden behind the tile's matrix work.
    static_assert(TD * 32 == 2 * NW * 64, "two float4s per thread per tile");
    const int q4 = tid & 31, r4 = tid >> 5;
    const float4 mq = *reinterpret_cast<const float4*>(pca_mean + 4 * q4);
    float4 pre[2];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int r = r4 + 16 * j;
            pre[j] = t0 + r < tend ? *reinterpret_cast<const float4*>(D + (int64_t)(t0 + r) * kDescDim + 4 * q4)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (tbeg < tend) fetch(tbeg);

    for (int t0 = tbeg; t0 < tend; t0 += TD) {
        __syncthreads();   // the previous tile's readers are done
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int r = r4 + 16 * j;
            const bool live = t0 + r < tend;
            float* d = Dl + r * DSTR + 4 * q4;
            d[0] = live ? pre[j].x - mq.x : 0.f;
            d[1] = live ? pre[j].y - mq.y : 0.f;
            d[2] = live ? pre[j].z - mq.z : 0.f;
            d[3] = live ? pre[j].w - mq.w : 0.f;
        }
        if (t0 + TD < tend) fetch(t0 + TD);
        __syncthreads();
        if (wave < 4) {
            // X tile (rows 16 rt.., cols 16 ct..) = Dl . A^T over k = 0..127
            const int rt = wave >> 1, ct = wave & 1;
            const float* arow = pca_matrix + (16 * ct + (lane & 15)) * kDescDim + (lane >> 4);
            const float* drow = Dl + (16 * rt + (lane & 15)) * DSTR + (lane >> 4);
            f4 x = f4{};
#pragma unroll 8
            for (int s = 0; s < 32; ++s) x = mfma16(drow[4 * s], arow[4 * s], x);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rt + 4 * (lane >> 4) + r, col = 16 * ct + (lane & 15);
                const float v = x[r], v2 = v * v;
                XXt[col * TD + row] = v;
                XXt[(32 + col) * TD + row] = v2;
                XXr[row * XRS + col] = v;
                XXr[row * XRS + 32 + col] = v2;
            }
        }
        __syncthreads();
        // logits of this wave's 64 components for the tile's 32 descriptors
        f16v L[2] = {f16v{}, f16v{}};
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            const float a = XXt[(2 * s + h) * TD + c32];
            L[0] = mfma32(a, bf[0][s], L[0]);
            L[1] = mfma32(a, bf[1][s], L[1]);
        }
        // softmax over all 512 components: per-wave max and sum of each
        // descriptor row, then combined across the waves
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float l0 = L[0][i] + cc[0], l1 = L[1][i] + cc[1];
            const float mx = half_max(fmaxf(l0, l1));
            const float e0 = __expf(l0 - mx), e1 = __expf(l1 - mx);
            L[0][i] = e0;
            L[1][i] = e1;
            const float sm = half_sum(e0 + e1);
            if (c32 == 0) {
                const int d = 8 * (i >> 2) + 4 * h + (i & 3);
                redm[wave][d] = mx;
                reds[wave][d] = sm;
            }
        }
        __syncthreads();
        if (tid < TD) {
            float M = redm[0][tid];
#pragma unroll
            for (int w = 1; w < NW; ++w) M = fmaxf(M, redm[w][tid]);
            float S = 0.f;
#pragma unroll
            for (int w = 0; w < NW; ++w) S += reds[w][tid] * __expf(redm[w][tid] - M);
            rowq[tid][0] = M;
            rowq[tid][1] = (t0 + tid < tend) ? 1.f / S : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int d = 8 * (i >> 2) + 4 * h + (i & 3);
            const float q = __expf(redm[wave][d] - rowq[d][0]) * rowq[d][1];
            L[0][i] *= q;
            L[1][i] *= q;
            s0[0] += L[0][i];
            s0[1] += L[1][i];
        }
        // S1 | S2 += Q^T [X | X.*X]: the descriptor (K) index of step i is
        // 8(i/4) + 4(l/32) + i%4 -- the rows this lane's Q registers hold
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int d = 8 * (i >> 2) + 4 * h + (i & 3);
            const float b1 = XXr[d * XRS + c32], b2 = XXr[d * XRS + 32 + c32];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                acc1[t] = mfma32(L[t][i], b1, acc1[t]);
                acc2[t] = mfma32(L[t][i], b2, acc2[t]);
            }
        }
    }

    // S0 per component (this lane's logit column), then either the sums of
    // this part to its partial block or the image's outputs
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const float v = s0[t] + __shfl_xor(s0[t], 32);
        if (h == 0) {
            if constexpr (SPLIT) partial[(int64_t)blockIdx.x * kScfvPartialFloats + CPW * wave + 32 * t + c32] = v;
            else s0s[CPW * wave + 32 * t + c32] = v;
        }
    }
    if constexpr (SPLIT) {
        float* P = partial + (int64_t)blockIdx.x * kScfvPartialFloats + NC;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int comp = CPW * wave + 32 * t + 8 * (i >> 2) + 4 * h + (i & 3);
                P[comp * PD + c32] = acc1[t][i];
                P[NC * PD + comp * PD + c32] = acc2[t][i];
            }
    } else {
        __syncthreads();
        scfv_output(img, K, wave, lane, s0s, acc1, acc2, means, vars, prep, gm_out, gv_out, delta_out, order_out,
                    bits_out, skey, sidx);
    }
}

// Adds up the partial blocks of images aggregated in `splits` parts, into
// each image's first block (in part order): 512 floats per workgroup, so
// the sums of one image are spread over 65 workgroups.
__global__ __launch_bounds__(256) void k_scfv_reduce(float* __restrict__ partial, int splits) {
    constexpr int kChunks = kScfvPartialFloats / 512;
    static_assert(kScfvPartialFloats % 512 == 0, "whole chunks");
    const int img = blockIdx.x / kChunks, chunk = blockIdx.x % kChunks;
    float* P0 = partial + (int64_t)img * splits * kScfvPartialFloats + chunk * 512;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int e = threadIdx.x + 256 * j;
        float a = P0[e];
        for (int p = 1; p < splits; ++p) a += P0[(int64_t)p * kScfvPartialFloats + e];
        P0[e] = a;
    }
}

// Completes images aggregated in parts whose sums k_scfv_reduce has put in
// each image's first partial block (blocks `splits` apart): writes the
// outputs as k_scfv does.
__global__ __launch_bounds__(512) void k_scfv_join(const float* __restrict__ partial, int splits,
                                                   const int32_t* __restrict__ count, int kp_cap,
                                                   const float* __restrict__ means, const float* __restrict__ vars,
                                                   const float* __restrict__ prep, float* __restrict__ gm_out,
                                                   float* __restrict__ gv_out, float* __restrict__ delta_out,
                                                   int32_t* __restrict__ order_out, uint32_t* __restrict__ bits_out) {
    __shared__ float s0s[NC];
    __shared__ float skey[NC];
    __shared__ int sidx[NC];
    const int img = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, h = lane >> 5, c32 = lane & 31;
    const int K = min(max(count[img], 0), kp_cap);
    const float* P0 = partial + (int64_t)img * splits * kScfvPartialFloats;
    s0s[tid] = P0[tid];
    f16v acc1[2], acc2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int comp = CPW * wave + 32 * t + 8 * (i >> 2) + 4 * h + (i & 3);
            acc1[t][i] = P0[NC + comp * PD + c32];
            acc2[t][i] = P0[NC + NC * PD + comp * PD + c32];
        }
    __syncthreads();
    scfv_output(img, K, wave, lane, s0s, acc1, acc2, means, vars, prep, gm_out, gv_out, delta_out, order_out,
                bits_out, skey, sidx);
}

}  // namespace

hipError_t launch_scfv(const float* desc, const int32_t* count, int n_images, int kp_cap, const float* pca_mean,
                       const float* pca_matrix, const float* weights, const float* means, const float* vars,
                       float* prep, float* gm, float* gv, float* delta, int32_t* order, uint32_t* bits,
                       hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scfv_prep, dim3(NC / 8), dim3(256), 0, s, weights, means, vars, prep);
    hipLaunchKernelGGL(k_scfv<false>, dim3(n_images), dim3(NW * 64), 0, s, desc, count, kp_cap, 1, 0, pca_mean,
                       pca_matrix, means, vars, prep, nullptr, gm, gv, delta, order, bits);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// The allocation-free form: its scratch is this file-scope array, one copy
// per GPU, looked up once per device with hipGetSymbolAddress.  In host
// code `scratch` names a host-side stand-in, never the device memory: only
// the looked-up address is passed to kernels.
static __device__ __align__(256) float scratch[kScfvStaticFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};
}  // namespace

int scfv_static_splits(int n_images, int kp_cap) {
    if (n_images <= 0 || n_images > kScfvStaticPartials / 2) return 1;
    const int tiles = (kp_cap + TD - 1) / TD;
    return std::max(1, std::min(tiles, kScfvStaticPartials / n_images));
}

hipError_t scfv_static_scratch(float** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

hipError_t launch_scfv_static(float* scr, int splits, const float* desc, const int32_t* count, int n_images,
                              int kp_cap, const float* pca_mean, const float* pca_matrix, const float* weights,
                              const float* means, const float* vars, float* gm, float* gv, float* delta,
                              int32_t* order, uint32_t* bits, hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    float* prep = scr;
    hipLaunchKernelGGL(k_scfv_prep, dim3(NC / 8), dim3(256), 0, s, weights, means, vars, prep);
    if (splits <= 1) {
        hipLaunchKernelGGL(k_scfv<false>, dim3(n_images), dim3(NW * 64), 0, s, desc, count, kp_cap, 1, 0, pca_mean,
                           pca_matrix, means, vars, prep, nullptr, gm, gv, delta, order, bits);
    } else {
        float* partial = scr + kScfvStaticPrepFloats;
        const int tiles = (kp_cap + TD - 1) / TD;
        const int per = (tiles + splits - 1) / splits;
        hipLaunchKernelGGL(k_scfv<true>, dim3(n_images * splits), dim3(NW * 64), 0, s, desc, count, kp_cap, splits,
                           per, pca_mean, pca_matrix, means, vars, prep, partial, nullptr, nullptr, nullptr, nullptr,
                           nullptr);
        hipLaunchKernelGGL(k_scfv_reduce, dim3(n_images * (kScfvPartialFloats / 512)), dim3(256), 0, s, partial,
                           splits);
        hipLaunchKernelGGL(k_scfv_join, dim3(n_images), dim3(NW * 64), 0, s, partial, splits, count, kp_cap, means,
                           vars, prep, gm, gv, delta, order, bits);
    }
    return hipGetLastError();
}

}  // namespace cdvs
