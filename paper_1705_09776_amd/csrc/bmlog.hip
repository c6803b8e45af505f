// BMLoG scale space on gfx950: the block-based mixture-domain variant the
// paper compares (Sec. III-A) -- Gaussian scale images filtered in the
// frequency domain block by block, the Laplacian left to the spatial
// detector -- built as an alternative to cdvs_pyramid with the same output
// layout, to measure it against the spatial filters on this GPU.
//
// One 512-lane workgroup per 128 x 128 block (blocks overlap by 16 pixels
// on every side and keep their central 96 x 96; pixels outside the octave
// image come from its nearest edge pixel), two workgroups per CU: one LDS
// work buffer of 128 rows x 64 complex (row stride 65), the block's
// spectrum held in registers (16 values per lane) across all its scales.
//
// Each 1-D transform is two passes of small DFTs held in registers, with
// one LDS exchange between them (Cooley-Tukey, N = N1 N2: a pass of
// N1-point DFTs along a stride, a twiddle, a pass of N2-point DFTs on
// contiguous runs):
//   forward rows: the real rows as 64-point complex DFTs of the packed pairs
//            (x[2n], x[2n+1]) (8 x 8), split in place into the spectra
//            X[0..64] of the real rows, X[0] and X[64] (both real) packed
//            as one complex value; then 128-point DFTs down the 64 columns
//            (8 x 16), the packed column giving X[.][0] + i X[.][64]
//            transformed, each lane keeping one 16-frequency run of one
//            column;
//   per output scale: the spectrum times the separable real transfer
//            function H(v) H(u) (the packed column takes H(0) and H(64)
//            apart through the Hermitian pair P(v), P(128 - v)), 128-point
//            inverse DFTs down the columns (16 x 8), the kept rows' packed
//            transforms rebuilt from their half spectra, 64-point inverse
//            DFTs (8 x 8) whose second pass writes the central 96 x 96
//            pixels straight from registers, scaled by 1 / (128 * 64) (the
//            last scale's even samples also to the next octave's base).
// Passes write back to the positions they read (no barrier inside them),
// except the forward rows' second pass, which reads, waits and writes its
// output in natural order so that the split works in place.  After the
// forward column passes frequency k1 + 8 k2 sits at position 16 k1 + k2;
// the inverse passes take that order and return natural order.  Lanes run
// over rows (or columns), so with the row stride of 65 complex the LDS
// accesses of a wave are conflict-free or at the two-cycle minimum of
// 64-bit accesses.
#include "cdvs_internal.h"

namespace cdvs {

namespace {

constexpr int BN = kBmN;        // 128
constexpr int BR = kBmR;        // 16
constexpr int BS = BN - 2 * BR; // 96
constexpr int HN = BN / 2;      // 64 complex per row (packed pairs / half spectrum)
constexpr int RS = HN + 1;      // LDS row stride, in complex values
constexpr int NT = 512;
static_assert(BN == 128 && BR == 16, "the pass plan is written for 128-point blocks");

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// b exp(-+2 pi i J / LEN) for compile-time J < LEN / 2, LEN <= 16 (INV: +),
// with the trivial twiddles 1 and -+i taken without multiplies.
template <int J, int LEN, bool INV>
__device__ __forceinline__ float2 twiddle_mul(float2 b) {
    static_assert(J < LEN / 2 && LEN <= 16, "twiddle");
    if constexpr (J == 0) {
        return b;
    } else if constexpr (4 * J == LEN) {
        return INV ? make_float2(-b.y, b.x) : make_float2(b.y, -b.x);
    } else {
        // cos and sin of 2 pi J / LEN = m pi / 8
        constexpr int m = J * (16 / LEN);   // 1..7, not 4
        constexpr float c1 = 0.92387953251128674f, c2 = 0.70710678118654752f, c3 = 0.38268343236508977f;
        constexpr float cs = m == 1 ? c1 : m == 2 ? c2 : m == 3 ? c3 : m == 5 ? -c3 : m == 6 ? -c2 : -c1;
        constexpr float sn = m == 1 ? c3 : m == 2 ? c2 : m == 3 ? c1 : m == 5 ? c1 : m == 6 ? c2 : c3;
        return cmul(b, make_float2(cs, INV ? sn : -sn));
    }
}

// Butterflies J, J+1, .. of every group of one radix-2 stage of span LEN.
template <int LEN, int J, bool INV, int N>
__device__ __forceinline__ void stage_from(float2 (&x)[N]) {
    if constexpr (J < LEN / 2) {
#pragma unroll
        for (int i = 0; i < N; i += LEN) {
            const float2 a = x[i + J], b = twiddle_mul<J, LEN, INV>(x[i + J + LEN / 2]);
            x[i + J] = cadd(a, b);
            x[i + J + LEN / 2] = csub(a, b);
        }
        stage_from<LEN, J + 1, INV>(x);
    }
}

template <int LEN, bool INV, int N>
__device__ __forceinline__ void stages_from(float2 (&x)[N]) {
    if constexpr (LEN <= N) {
        stage_from<LEN, 0, INV>(x);
        stages_from<2 * LEN, INV>(x);
    }
}

// In-register N-point DFT (N = 8 or 16), natural order in and out,
// unnormalised; forward exp(-2 pi i nk / N), INV exp(+2 pi i nk / N):
// radix-2 decimation in time on the bit-reversed input (a renaming of
// registers).
template <int N, bool INV>
__device__ __forceinline__ void dft(float2 (&x)[N]) {
    static_assert(N == 8 || N == 16, "dft size");
    constexpr int LG = N == 8 ? 3 : 4;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        int r = 0;
#pragma unroll
        for (int b = 0; b < LG; ++b) r |= ((i >> b) & 1) << (LG - 1 - b);
        if (i < r) {
            const float2 t = x[i];
            x[i] = x[r];
            x[r] = t;
        }
    }
    stages_from<2, INV>(x);
}

// One block of one octave: U8 = octave 0 (input the u8 image; outputs
// G_{0,0..4} through H rows 0 and 5..8), else input G_{o,0} and outputs
// G_{o,1..4} through H rows 1..4.
template <bool U8>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_bmlog(const uint8_t* __restrict__ images, float* __restrict__ pyr,
                                              const OctJob* __restrict__ jobs, const int32_t* __restrict__ blocks,
                                              const float* __restrict__ Ht) {
    constexpr int NOUT = U8 ? 5 : 4;
    __shared__ float2 W[BN * RS];   // work buffer
    __shared__ float2 P0[BN];       // spectrum of the packed column, by storage row
    __shared__ float2 tw[BN];       // exp(-2 pi i j / 128)
    __shared__ float Hs[NOUT][BN];  // the transfer functions applied here

    const int t = threadIdx.x;
    const int* blk = blocks + 3 * blockIdx.x;
    const OctJob& job = jobs[blk[0]];
    const int bx = blk[1], by = blk[2];
    const int w = job.w, h = job.h;
    const int x0 = bx * BS - BR, y0 = by * BS - BR;   // image position of block pixel (0, 0)

    if (t < BN) {
        float sn, cs;
        sincospif((float)t / 64.f, &sn, &cs);
        tw[t] = make_float2(cs, -sn);
    }
    for (int e = t; e < NOUT * BN; e += NT) {
        const int q = e / BN;
        Hs[q][e % BN] = Ht[(U8 ? (q == 0 ? 0 : 4 + q) : 1 + q) * BN + e % BN];
    }
    // block pixels as packed pairs in natural order (coalesced along rows)
#pragma unroll 4
    for (int j = 0; j < BN * HN / NT; ++j) {
        const int e = t + j * NT, r = e / HN, n = e % HN;
        const int gy = min(max(y0 + r, 0), h - 1);
        const int ga = min(max(x0 + 2 * n, 0), w - 1), gb = min(max(x0 + 2 * n + 1, 0), w - 1);
        float va, vb;
        if constexpr (U8) {
            const uint8_t* row = images + job.src + (int64_t)gy * job.src_pitch;
            va = (float)row[ga];
            vb = (float)row[gb];
        } else {
            const float* row = pyr + job.plane0 + (int64_t)gy * job.pitch;
            va = row[ga];
            vb = row[gb];
        }
        W[r * RS + n] = make_float2(va, vb);
    }
    __syncthreads();

    // forward rows, pass 1: task (row r, n2): z[n2 + 8 n1] -> 8-point DFT
    // over n1 -> times w64^(n2 k1) -> position n2 + 8 k1
#pragma unroll
    for (int j = 0; j < BN * 8 / NT; ++j) {
        const int e = t + j * NT, r = e % BN, n2 = e / BN;
        float2 x[8];
        float2* row = W + r * RS + n2;
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = row[8 * i];
        dft<8, false>(x);
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) row[8 * k1] = k1 == 0 ? x[0] : cmul(x[k1], tw[(2 * n2 * k1) & (BN - 1)]);
    }
    __syncthreads();
    // pass 2: task (r, k1): positions 8 k1 .. 8 k1 + 7 -> 8-point DFT ->
    // Z[k1 + 8 k2], written in natural order once every task has read
    {
        constexpr int NJ = BN * 8 / NT;
        float2 x[NJ][8];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int e = t + j * NT, r = e % BN, k1 = e / BN;
            const float2* run = W + r * RS + 8 * k1;
#pragma unroll
            for (int i = 0; i < 8; ++i) x[j][i] = run[i];
            dft<8, false>(x[j]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int e = t + j * NT, r = e % BN, k1 = e / BN;
            float2* row = W + r * RS + k1;
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) row[8 * k2] = x[j][k2];
        }
    }
    __syncthreads();
    // split each row's packed transform Z into the spectrum of the real row,
    // in place: E = (Z[k] + conj Z[64-k]) / 2, O = (Z[k] - conj Z[64-k]) / 2i,
    // X[k] = E + w^k O, X[64-k] = conj E - conj(w^k) conj O
    // (w = exp(-2 pi i / 128)); X[0] + i X[64] at position 0
#pragma unroll 2
    for (int j = 0; j < BN * 32 / NT; ++j) {
        const int e = t + j * NT, r = e % BN, k = e / BN;   // k = 0 also does k = 32
        float2* X = W + r * RS;
        if (k == 0) {
            const float2 z0 = X[0], z32 = X[32];
            X[0] = make_float2(z0.x + z0.y, z0.x - z0.y);
            // k = 32 pairs with itself: E = Re z, O = Im z, w^32 = -i
            X[32] = make_float2(z32.x, -z32.y);
        } else {
            const float2 zk = X[k], zm = X[HN - k];
            const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            const float2 O = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            const float2 wk = tw[k];
            X[k] = cadd(E, cmul(wk, O));
            X[HN - k] = csub(conjf2(E), cmul(conjf2(wk), conjf2(O)));
        }
    }
    __syncthreads();
    // forward columns, pass 1: task (column u, n2): rows 16 n1 + n2 ->
    // 8-point DFT over n1 -> times w128^(n2 k1) -> rows 16 k1 + n2
#pragma unroll
    for (int j = 0; j < HN * 16 / NT; ++j) {
        const int e = t + j * NT, u = e % HN, n2 = e / HN;
        float2 x[8];
        float2* col = W + n2 * RS + u;
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = col[16 * i * RS];
        dft<8, false>(x);
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) col[16 * k1 * RS] = k1 == 0 ? x[0] : cmul(x[k1], tw[(n2 * k1) & (BN - 1)]);
    }
    __syncthreads();
    // pass 2: task (u, k1) = this thread: rows 16 k1 .. 16 k1 + 15 ->
    // 16-point DFT -> frequencies v = k1 + 8 k2, kept in registers for every
    // output scale (the packed column also in P0, for its Hermitian pairs)
    static_assert(HN * 8 == NT, "one spectrum run per thread");
    const int u = t % HN, k1 = t / HN;
    float2 spec[16];
    {
        const float2* col = W + 16 * k1 * RS + u;
#pragma unroll
        for (int i = 0; i < 16; ++i) spec[i] = col[i * RS];
        dft<16, false>(spec);
        if (u == 0) {
#pragma unroll
            for (int k2 = 0; k2 < 16; ++k2) P0[16 * k1 + k2] = spec[k2];
        }
    }
    __syncthreads();

    // unnormalised transforms: 128-point columns, then 64-point packed rows
    const float scale = 1.f / (float)(BN * HN);
    for (int q = 0; q < NOUT; ++q) {
        const float* H = Hs[q];
        // inverse columns, pass A: the filtered spectrum run (frequency
        // v = k1 + 8 k2) -> 16-point inverse DFT over k2 -> rows 16 k1 + n2
        // of W.  The packed column holds P = F0 + i F64 (F0, F64 the
        // Hermitian transforms of the real columns 0 and 64); filtered, it is
        // H(v) (a P(v) + b conj P(128 - v)), a = (H(0) + H(64)) / 2,
        // b = (H(0) - H(64)) / 2, P(128 - v) sitting at storage row
        // 16 ((8 - k1) & 7) + ((16 - k2 - (k1 != 0)) & 15), which is
        // pb - k2 with pb = 16 ((8 - k1) & 7) + 15 + (k1 == 0), except row 0
        // for k1 = k2 = 0.
        {
            float2 x[16];
            if (u != 0) {
                const float hu = H[u];
#pragma unroll
                for (int k2 = 0; k2 < 16; ++k2) x[k2] = cscale(spec[k2], H[k1 + 8 * k2] * hu);
            } else {
                const float a = 0.5f * (H[0] + H[HN]), b = 0.5f * (H[0] - H[HN]);
                const int pb = 16 * ((8 - k1) & 7) + 15 + (k1 == 0);
#pragma unroll
                for (int k2 = 0; k2 < 16; ++k2) {
                    const float2 p = spec[k2], pm = P0[k2 == 0 && k1 == 0 ? 0 : pb - k2];
                    const float hv = H[k1 + 8 * k2];
                    x[k2] = make_float2(hv * (a * p.x + b * pm.x), hv * (a * p.y - b * pm.y));
                }
            }
            dft<16, true>(x);
            float2* out = W + 16 * k1 * RS + u;
#pragma unroll
            for (int n2 = 0; n2 < 16; ++n2) out[n2 * RS] = x[n2];
        }
        __syncthreads();
        // pass B: task (u, n2): rows 16 k1 + n2 times conj w128^(n2 k1) ->
        // 8-point inverse DFT over k1 -> block row 16 n1 + n2
#pragma unroll 1
        for (int j = 0; j < HN * 16 / NT; ++j) {
            const int e = t + j * NT, uu = e % HN, n2 = e / HN;
            float2 x[8];
            float2* col = W + n2 * RS + uu;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                x[kk] = kk == 0 ? col[0] : cmulc(col[16 * kk * RS], tw[(n2 * kk) & (BN - 1)]);
            dft<8, true>(x);
#pragma unroll
            for (int n1 = 0; n1 < 8; ++n1) col[16 * n1 * RS] = x[n1];
        }
        __syncthreads();
        // rebuild each kept row's packed transform (natural order) from its
        // half spectrum: E = (X[k] + conj X[64-k]) / 2,
        // O = (X[k] - conj X[64-k]) conj(w^k) / 2, Z[k] = E + i O
#pragma unroll 2
        for (int j = 0; j < BS * 32 / NT; ++j) {
            const int e = t + j * NT, r = BR + e % BS, k = e / BS;   // k = 0 also does k = 32
            float2* X = W + r * RS;
            if (k == 0) {
                // X[0] = X[0].x and X[64] = X[0].y, both real (w^0 = 1);
                // X[32] pairs with itself (conj(w^32) = i)
                const float2 x0 = X[0], x32 = X[32];
                X[0] = make_float2(0.5f * (x0.x + x0.y), 0.5f * (x0.x - x0.y));
                X[32] = make_float2(x32.x, -x32.y);
            } else {
                const float2 xk = X[k], xm = X[HN - k];
                const float2 wk = tw[k];
                const float2 E = make_float2(0.5f * (xk.x + xm.x), 0.5f * (xk.y - xm.y));
                const float2 O = cmulc(make_float2(0.5f * (xk.x - xm.x), 0.5f * (xk.y + xm.y)), wk);
                X[k] = make_float2(E.x - O.y, E.y + O.x);
                // for 64 - k: E' = conj E, O' = (X[64-k] - conj X[k]) conj(w^(64-k)) / 2,
                // conj(w^(64-k)) = -w^k
                const float2 O2 = cmul(make_float2(0.5f * (xm.x - xk.x), 0.5f * (xm.y + xk.y)),
                                       make_float2(-wk.x, -wk.y));
                X[HN - k] = make_float2(E.x - O2.y, -E.y + O2.x);
            }
        }
        __syncthreads();
        // inverse rows, pass 1: task (r, k2): positions 8 k1 + k2 -> 8-point
        // inverse DFT over k1 -> times conj w64^(n1 k2) -> position 8 n1 + k2
        for (int e = t; e < BS * 8; e += NT) {
            const int r = BR + e % BS, k2 = e / BS;
            float2 x[8];
            float2* row = W + r * RS + k2;
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = row[8 * i];
            dft<8, true>(x);
#pragma unroll
            for (int n1 = 0; n1 < 8; ++n1)
                row[8 * n1] = n1 == 0 ? x[0] : cmulc(x[n1], tw[(2 * n1 * k2) & (BN - 1)]);
        }
        __syncthreads();
        // pass 2: task (n1, r), n1 fastest over the lanes: positions 8 n1 ..
        // 8 n1 + 7 -> 8-point inverse DFT over k2 -> z[n1 + 8 n2] = the pixel
        // pair at block columns 2 n, 2 n + 1 (n = n1 + 8 n2); the kept
        // columns 16..111 are n2 = 1..6
        const int plane = U8 ? q : q + 1;   // G_{o,plane}
        for (int e = t; e < BS * 8; e += NT) {
            const int n1 = e % 8, r = BR + e / 8;
            float2 x[8];
            const float2* run = W + r * RS + 8 * n1;
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = run[i];
            dft<8, true>(x);
            const int gy = y0 + r;
            const bool down = job.next0 >= 0 && q == NOUT - 1 && (gy & 1) == 0;
            if (gy < h) {
                float* out = pyr + job.plane0 + (int64_t)plane * job.plane_stride + (int64_t)gy * job.pitch;
#pragma unroll
                for (int n2 = 1; n2 < 7; ++n2) {
                    const int gx = x0 + 2 * (n1 + 8 * n2);
                    if (gx >= w) continue;
                    // (plain stores: this kernel's 8-byte stores cover half
                    // lines, which non-temporal stores wrote back 1.47x over)
                    const float a = x[n2].x * scale, b = x[n2].y * scale;
                    if (gx + 1 < w) *reinterpret_cast<float2*>(out + gx) = make_float2(a, b);
                    else out[gx] = a;
                    if (down) pyr[job.next0 + (int64_t)(gy >> 1) * job.next_pitch + (gx >> 1)] = a;
                }
            }
        }
        __syncthreads();   // W is rewritten by the next scale
    }
}

}  // namespace

hipError_t launch_bmlog(const uint8_t* images, float* pyr, const OctJob* jobs, const int32_t* blocks, int nblocks,
                        const float* H, bool octave0, hipStream_t stream) {
    if (nblocks <= 0) return hipSuccess;
    if (octave0)
        hipLaunchKernelGGL(k_bmlog<true>, dim3(nblocks), dim3(NT), 0, stream, images, pyr, jobs, blocks, H);
    else
        hipLaunchKernelGGL(k_bmlog<false>, dim3(nblocks), dim3(NT), 0, stream, images, pyr, jobs, blocks, H);
    return hipGetLastError();
}

}  // namespace cdvs
