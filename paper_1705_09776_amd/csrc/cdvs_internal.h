// Internal declarations of the gfx950 CDVS library: device tables, kernel
// parameter blocks and launchers.  Included by the library's own sources
// only; the public interface is include/cdvs.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "cdvs.h"

namespace cdvs {

// Scale space of the compiled kernels: sigma0 = 1.6, S = 4, five images per
// octave; direct blur sigmas s_0 = 1.6 (input pre-blur) and
// s_k = 1.6 sqrt(2^(k/2) - 1), k = 1..4, truncated at ceil(4 s).
constexpr int kScales = 5;
constexpr int kR0 = 7, kR1 = 5, kR2 = 7, kR3 = 9, kR4 = 12;
constexpr int kMaxR = 12;
constexpr int kTapStride = 2 * kMaxR + 1;  // 25
constexpr int kOriBins = 36;
constexpr int kMaxOri = 4;
constexpr int kDescDim = 128;
constexpr int kMaxOctaves = 16;
constexpr int kCandCap = 8192;  // pre-deduplication candidates per image

// Row pitch of every pyramid plane, in floats.
constexpr int kPitchAlign = 32;

// Gaussian taps g_k[p], p = -r_k..r_k, stored at g[k][p + r_k].
struct Taps {
    float g[kScales][kTapStride];
};

// One (image, octave) unit of work.
struct OctJob {
    int64_t plane0;    // float offset of G_{o,0} in the pyramid buffer
    int64_t next0;     // float offset of G_{o+1,0}, or -1 for the last octave
    int64_t src;       // byte offset of the u8 image (used at octave 0)
    int32_t w, h;      // octave size
    int32_t pitch;     // floats
    int32_t plane_stride;  // floats between G_{o,k} and G_{o,k+1}
    int32_t next_w, next_h, next_pitch;
    int32_t src_pitch;  // bytes
    int32_t image;
    int32_t octave;
    int32_t tiles_x_blur[5], tile0_blur[5];  // tiling of the blur kernels, per tile shape (kBlurTilings)
};

// One detection strip: everything the detection kernel needs to load and
// label it, so that a strip costs one record load (no job search).
struct DetTile {
    int64_t plane0;        // float offset of G_{o,0}
    int32_t plane_stride;  // floats between G_{o,k} and G_{o,k+1}
    int32_t pitch;         // floats
    int32_t w, h;          // octave size
    int32_t tx0, ty0;      // the strip's first centre (octave pixels)
    int32_t image, octave;
    int32_t cand_cap;      // the image's candidate capacity
    int32_t cand_blk;      // the image's first candidate slot / kCandBlock
};
static_assert(sizeof(DetTile) == 48, "DetTile is three 16-byte chunks");
constexpr int kCandBlock = 256;   // candidate regions start on multiples of this many records

// Per-image octave geometry for the keypoint kernels.
struct OctGeom {
    int64_t plane0;
    int32_t w, h, pitch, plane_stride;
};

struct DetParams {
    // alpha_i = sum_k beta[k][i] L_k with L_k = sigma_k^2 lap_k, taken as
    // sum_k bsig[k][i] lap_k: bsig[k][i] = sigma_k^2 beta[k][i] (octave units)
    float bsig[kScales][4];
    float lo, hi;            // extremal scale range [sigma_0, sigma_4)
    float contrast;
    float edge_lim;          // (r+1)^2 / r
    float max_off;
    int32_t border;
};

// Division of an unsigned 32-bit n by a fixed d >= 1 as a multiply-high and
// shifts (the round-up method of Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994): with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1 and t = mulhi(m, n), the quotient is
// (t + ((n - t) >> 1)) >> (l - 1) for every n < 2^32 (d = 1: n itself).
// The keypoint kernels take their (image, keypoint) slot apart with it in
// scalar registers.
struct KpDiv {
    uint32_t d, m;
    int32_t sh;   // l - 1; unused when d = 1
};

inline KpDiv make_kp_div(uint32_t d) {
    KpDiv v{d, 0u, 0};
    if (d > 1) {
        int l = 0;
        while ((1ull << l) < d) ++l;
        v.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1ull);
        v.sh = l - 1;
    }
    return v;
}

__device__ __forceinline__ uint32_t kp_div_q(uint32_t n, const KpDiv& v) {
    if (v.d == 1u) return n;
    const uint32_t t = __umulhi(v.m, n);
    return (t + ((n - t) >> 1)) >> v.sh;
}

struct OriParams {
    float radius, wsigma, peak;
    float sigma0;
    float fix;      // fixed-point scale of the LDS histogram (a power of two)
    float inv_fix;  // 1 / fix, exact
    float lfix;     // log2(fix), an integer
    int32_t max_ori;
    int32_t kp_cap;
    KpDiv kp_div;   // division of a keypoint slot by kp_cap
};

struct DescParams {
    float cell, radius, wsigma, clamp;
    float sigma0;
    float fix;      // fixed-point scale of the LDS histogram (a power of two)
    float inv_fix;  // 1 / fix, exact
    float lfix;     // log2(fix), an integer
    int32_t kp_cap;
    KpDiv kp_div;
};

// Workgroups are dealt to the 8 XCDs of an MI355X round-robin by block
// index, and each XCD has its own L2.  xcd_remap turns block b of a grid of n
// into a logical index such that every XCD walks one contiguous range of
// tiles (neighbouring tiles share halo rows and columns through that XCD's
// L2).  It is a bijection on [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int x = b % kXcds, i = b / kXcds;
    const int per = n / kXcds, rem = n % kXcds;
    return x * per + min(x, rem) + i;
}

// The value held by lane ^ S of the wave, for a compile-time S < 64: row
// operations (DPP) for S = 1, 2, the swizzle's bit-mask mode (within 32
// lanes) for S = 4, 8, 16, and a lane permute for 32.  Every lane must be
// active.
template <int S>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    static_assert(S > 0 && S < 64 && (S & (S - 1)) == 0, "a power of two below 64");
    if constexpr (S == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xf, 0xf, false);
    else if constexpr (S == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xf, 0xf, false);
    else if constexpr (S <= 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (S << 10) | 0x1F);
    else return (uint32_t)__shfl_xor((int)v, S);
}
template <int S>
__device__ __forceinline__ unsigned long long lane_xor64(unsigned long long v) {
    return ((unsigned long long)lane_xor<S>((uint32_t)(v >> 32)) << 32) | lane_xor<S>((uint32_t)v);
}

// Bits of the device status word.
constexpr int kFlagCandOverflow = 1;
constexpr int kFlagSelectInexact = 2;   // a reduced image's top-k reached its selection threshold
constexpr int kFlagFrontShape = 4;      // a front-end source image does not map onto the context's image

// Surrogate CNN geometry: one entry per image.
constexpr int kCnnChannels = 16, kCnnHeads = 6, kCnnLayers = 4;
constexpr int kCnnParams = kCnnLayers * (9 * 16 * 16 + 16) + 16 * 6 + 6;  // 9382
constexpr int kCnnTileW = 16, kCnnTileH = 4;  // cells per conv workgroup
constexpr int kCnnFusedW = 32, kCnnFusedH = 16;  // output cells per fused-inference workgroup
struct CnnImage {
    int64_t cell0;     // first cell of the image in the batch's cell arrays
    int64_t src;       // byte offset of the u8 image
    int32_t src_pitch, H, W;
    int32_t H4, W4;    // grid of 4x4 cells
    int32_t n_oct;     // octaves of the image (valid head channels)
    int32_t tiles_x;   // 16-cell segments per row
    int32_t tile0;     // first conv tile (16 x 4 cells) of the image
    int32_t chunk0;    // first 16-cell row chunk of the image
    int32_t ftiles_x;  // fused-inference tiles (kCnnFusedW x kCnnFusedH cells) per row
    int32_t ftile0;    // first fused-inference tile of the image
};

// Gating of detection by a cell mask.
struct GateParams {
    const uint8_t* mask;     // per cell, bit o = octave o active; nullptr = plain
    const int32_t* active;   // [image][kMaxOctaves] active cells of the mask
    const CnnImage* cells;   // per image cell grid
    float fmax;              // fraction of active cells above which detection is dense
};

// Kernel tile shapes (width x height).  Shapes 0..3 are the scale-plane
// kernel's variants (autotuned); shape 4 is the pre-blur's own, 128 x 32
// (measured against 64 x 32, 80 x 32, 160 x 16 and 160 x 32: its column
// windows and row groups fill the workgroup's lanes best).
constexpr int kBlurVariants = 4;
constexpr int kPreblurVariant = 4;
constexpr int kBlurTilings = 5;
constexpr int kBlurV = 8;
__host__ __device__ constexpr int blur_tw(int v) { return v == 1 || v == 4 ? 128 : v == 2 ? 32 : 64; }
__host__ __device__ constexpr int blur_th(int v) { return v == 1 || v == 3 ? 16 : 32; }
static_assert(sizeof(OctJob::tiles_x_blur) / sizeof(int32_t) == kBlurTilings, "one tiling per blur tile shape");

// Launchers (each enqueues on `stream`, returns the launch error).
hipError_t launch_preblur(const uint8_t* images, float* pyr, const OctJob* jobs, const int32_t* owner, int ntiles,
                          const Taps& taps, hipStream_t stream);
hipError_t launch_scales(float* pyr, const OctJob* jobs, const int32_t* owner, int ntiles, int variant,
                         const Taps& taps, hipStream_t stream);
hipError_t launch_clear(int32_t* p, int n, hipStream_t stream);
// Detection over strips of 60 x kDetStripH centres inside the detection
// border (tx0, ty0 = the strip's first centre), one wave at a time each;
// gated by gate.mask unless it is null.
constexpr int kDetStripW = 60, kDetStripH = 48;
// Launch forms (the detection's tunable variant): one wave per strip, or
// persistent: `grid` workgroups (rounded to a multiple of 8) pulling strips
// from per-XCD counters work[0..7], which must be zero at launch.
constexpr int kDetectPerStrip = 0, kDetectPersistent = 1, kDetectVariants = 2;
hipError_t launch_detect_strips(const float* pyr, const DetTile* strips, int nstrips, int variant, int grid,
                                const DetParams& dp, const GateParams& gate, int32_t* work, cdvs_keypoint* cand,
                                int32_t* cand_cnt, int32_t* flags, hipStream_t stream);
hipError_t launch_select(const cdvs_keypoint* cand, const int32_t* cand_cnt, const int64_t* cand_off,
                         const int32_t* cand_capv, int n_images, cdvs_keypoint* sel, hipStream_t stream);
hipError_t launch_finalize(const cdvs_keypoint* cand, const int32_t* cand_cnt, const int64_t* cand_off,
                           const int32_t* cand_capv, const cdvs_keypoint* sel, int n_images, float dedup_ratio,
                           int topk, int kp_cap, cdvs_keypoint* kp, int32_t* count, int32_t* flags,
                           hipStream_t stream);
hipError_t launch_orient(const float* pyr, const OctGeom* geom, const cdvs_keypoint* kp, const int32_t* count,
                         int n_images, const OriParams& op, cdvs_keypoint* ori, int32_t* ori_cnt,
                         hipStream_t stream);
hipError_t launch_orient_compact(const cdvs_keypoint* ori, const int32_t* ori_cnt, const int32_t* count_in,
                                 int n_images, int kp_cap, int topk, cdvs_keypoint* out, int32_t* count_out,
                                 hipStream_t stream);
hipError_t launch_describe(const float* pyr, const OctGeom* geom, const cdvs_keypoint* kp, const int32_t* count,
                           int n_images, const DescParams& dp, float* desc, hipStream_t stream);

constexpr int kCnnFragShorts = kCnnLayers * 5 * 64 * 8;   // packed MFMA weight fragments (5 tap pairs)
hipError_t launch_cnn_infer(const uint8_t* images, const float* params, short* frag, const CnnImage* imgs,
                            const int32_t* owner, int ntiles, float* logits, uint8_t* mask, float zthr, hipStream_t s);
hipError_t launch_cnn_forward(const uint8_t* images, const float* params, short* acts, int64_t ncells,
                              const CnnImage* imgs, int nimg, int ntiles, float* logits, uint8_t* mask, float zthr,
                              hipStream_t s);
hipError_t launch_cnn_backward(const uint8_t* images, const float* params, const short* acts, int64_t ncells,
                               const CnnImage* imgs, int nimg, int ntiles, int nchunks, const float* logits,
                               const uint32_t* labels, const float* pos_w, short* dbuf, float* grad, float* loss,
                               int wgrid, hipStream_t s);
hipError_t launch_cnn_adam(float* p, const float* g, float* m, float* v, int step, float lr, float b1, float b2,
                           float eps, hipStream_t s);
hipError_t launch_cnn_labels(const cdvs_keypoint* kp, const int32_t* count, int kp_cap, const CnnImage* imgs, int nimg,
                             int64_t ncells, uint32_t* labels, hipStream_t s);
hipError_t launch_mask_count(const uint8_t* mask, const CnnImage* imgs, int nimg, int32_t* active, hipStream_t s);

// SCFV aggregation: 512 components of 32 dimensions; per-call constants
// derived from the model (B = [M./V, -1/(2V)] per component, c, 1/sqrt(w),
// 1/sigma) at these float offsets of a scratch block of kScfvPrepFloats.
constexpr int kScfvComponents = 512, kScfvDim = 32;
constexpr int kScfvPrepB = 0;
constexpr int kScfvPrepC = kScfvPrepB + kScfvComponents * 64;
constexpr int kScfvPrepRsw = kScfvPrepC + kScfvComponents;
constexpr int kScfvPrepIsig = kScfvPrepRsw + kScfvComponents;
constexpr int kScfvPrepFloats = kScfvPrepIsig + kScfvComponents * kScfvDim;   // 50176
hipError_t launch_scfv(const float* desc, const int32_t* count, int n_images, int kp_cap, const float* pca_mean,
                       const float* pca_matrix, const float* weights, const float* means, const float* vars,
                       float* prep, float* gm, float* gv, float* delta, int32_t* order, uint32_t* bits,
                       hipStream_t s);
// The allocation-free form keeps the same constants and, for small
// batches, per-part sums S0, S1, S2 (kScfvPartialFloats each) of images
// split into parts, in one file-scope device array per GPU: the constants
// first, then kScfvStaticPartials partial blocks.
constexpr int kScfvPartialFloats = kScfvComponents * (1 + 2 * kScfvDim);                   // 33280
constexpr int kScfvStaticPartials = 64;
constexpr int kScfvStaticPrepFloats = (kScfvPrepFloats + 63) / 64 * 64;
constexpr int64_t kScfvStaticFloats = kScfvStaticPrepFloats + (int64_t)kScfvStaticPartials * kScfvPartialFloats;
// Parts per image for a batch: 1 (one workgroup per image, no partial sums)
// unless the batch is at most half the partial blocks, then as many parts
// as fit, at most one per 32-descriptor tile.
int scfv_static_splits(int n_images, int kp_cap);
// Device address of this GPU's array (looked up once per device).
hipError_t scfv_static_scratch(float** out);
hipError_t launch_scfv_static(float* scr, int splits, const float* desc, const int32_t* count, int n_images,
                              int kp_cap, const float* pca_mean, const float* pca_matrix, const float* weights,
                              const float* means, const float* vars, float* gm, float* gv, float* delta,
                              int32_t* order, uint32_t* bits, hipStream_t s);

// Keypoint relevance: five characteristics, 15 bin edges and 16 table
// values each.
constexpr int kRelFeatures = 5, kRelEdges = 15, kRelBins = 16;
hipError_t launch_relevance(const cdvs_keypoint* kp_in, const int32_t* count_in, const int32_t* wh, int n_images,
                            int kp_cap, const float* edges, const float* values, int n_keep, cdvs_keypoint* kp_out,
                            int32_t* count_out, float* score_out, hipStream_t s);

// BMLoG scale space (the block frequency-domain variant): blocks of kBmN
// pixels overlapping by kBmR on every side, one (job, bx, by) triple per
// block; kBmTransfers rows of kBmN transfer-function values (g0, g1..g4,
// then g0 g1 .. g0 g4).
constexpr int kBmN = 128, kBmR = 16, kBmStep = kBmN - 2 * kBmR, kBmTransfers = 9;
hipError_t launch_bmlog(const uint8_t* images, float* pyr, const OctJob* jobs, const int32_t* blocks, int nblocks,
                        const float* H, bool octave0, hipStream_t stream);

// Front end: longer side brought down to kFrontLongSide; the output size
// (the longer side 640, the shorter rounded half up, at least 1; images
// already within 640 unchanged).  Host and device share this rule.
constexpr int kFrontLongSide = 640;
__host__ __device__ inline void front_size(int w, int h, int* ow, int* oh) {
    const int L = w > h ? w : h;
    if (L <= kFrontLongSide) {
        *ow = w;
        *oh = h;
        return;
    }
    const int sw = (2 * kFrontLongSide * w + L) / (2 * L), sh = (2 * kFrontLongSide * h + L) / (2 * L);
    *ow = sw > 1 ? sw : 1;
    *oh = sh > 1 ? sh : 1;
}
hipError_t launch_front(const uint8_t* src, const cdvs_image_desc* sdesc, uint8_t* dst,
                        const cdvs_image_desc* ddesc, int n, int32_t* flags, hipStream_t s);

// Transform coding and ternary quantisation: eight code words per descriptor.
constexpr int kTqWords = 8;
hipError_t launch_tq_encode(const float* desc, const int32_t* count, int n_images, int kp_cap, const float* lo,
                            const float* hi, const int32_t* order, int n_elem, uint32_t* codes, hipStream_t s);

}  // namespace cdvs
