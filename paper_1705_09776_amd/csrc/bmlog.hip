// BMLoG scale space on gfx950: the block-based mixture-domain variant the
// paper compares (Sec. III-A) -- Gaussian scale images filtered in the
// frequency domain block by block, the Laplacian left to the spatial
// detector -- built as an alternative to cdvs_pyramid with the same output
// layout, to measure it against the spatial filters on this GPU.
//
// One 256-lane workgroup per 128 x 128 block (blocks overlap by 16 pixels on
// every side and keep their central 96 x 96; pixels outside the octave
// image come from its nearest edge pixel).  The block's spectrum and a work
// buffer, 128 rows x 65 complex each (the half spectrum of real rows),
// stay in LDS:
//   forward: rows as 64-point complex FFTs of the packed pairs
//            (x[2n], x[2n+1]), split into the 65-bin spectra of the real
//            rows; then 128-point FFTs down the 65 columns;
//   per output scale: the spectrum times the separable real transfer
//            function H(v) H(u) into the work buffer, 128-point inverse FFTs
//            down the columns, the real rows rebuilt from their half spectra
//            as 64-point inverse FFTs, scaled by 1 / (128 * 64), and the
//            central 96 x 96 pixels written out (the last scale's even
//            samples also to the next octave's base).
// Radix-2 decimation-in-time FFTs in place, input in bit-reversed order,
// twiddles exp(-2 pi i j / 128) from an LDS table.
#include "cdvs_internal.h"

namespace cdvs {

namespace {

constexpr int BN = kBmN;        // 128
constexpr int BR = kBmR;        // 16
constexpr int BS = BN - 2 * BR; // 96
constexpr int HC = BN / 2 + 1;  // 65: half-spectrum columns (row stride of the LDS buffers)
constexpr int NT = 256;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ int rev6(int n) { return (int)(__brev((unsigned)n) >> 26); }
__device__ __forceinline__ int rev7(int n) { return (int)(__brev((unsigned)n) >> 25); }

// 64-point FFTs along each of the 128 rows (elements 0..63 of a row),
// input bit-reversed, in place; INV: conjugate twiddles (no scaling).
template <bool INV>
__device__ __forceinline__ void rows_fft64(float2* A, const float2* tw) {
#pragma unroll 1
    for (int s = 0; s < 6; ++s) {
        const int half = 1 << s;
        for (int it = threadIdx.x; it < BN * 32; it += NT) {
            const int row = it >> 5, j = it & 31;
            const int pos = j & (half - 1), i0 = ((j >> s) << (s + 1)) + pos, i1 = i0 + half;
            float2 w = tw[pos << (6 - s)];
            if (INV) w.y = -w.y;
            float2* x = A + row * HC;
            const float2 a = x[i0], b = cmul(x[i1], w);
            x[i0] = cadd(a, b);
            x[i1] = csub(a, b);
        }
        __syncthreads();
    }
}

// 128-point FFTs down each of the 65 columns, input bit-reversed along the
// rows, in place.
template <bool INV>
__device__ __forceinline__ void cols_fft128(float2* A, const float2* tw) {
#pragma unroll 1
    for (int s = 0; s < 7; ++s) {
        const int half = 1 << s;
        for (int it = threadIdx.x; it < HC * 64; it += NT) {
            const int j = it / HC, col = it - j * HC;
            const int pos = j & (half - 1), i0 = ((j >> s) << (s + 1)) + pos, i1 = i0 + half;
            float2 w = tw[pos << (6 - s)];
            if (INV) w.y = -w.y;
            const float2 a = A[i0 * HC + col], b = cmul(A[i1 * HC + col], w);
            A[i0 * HC + col] = cadd(a, b);
            A[i1 * HC + col] = csub(a, b);
        }
        __syncthreads();
    }
}

// One block of one octave: U8 = octave 0 (input the u8 image; outputs
// G_{0,0..4} through H rows 0 and 5..8), else input G_{o,0} and outputs
// G_{o,1..4} through H rows 1..4.
template <bool U8>
__global__ __launch_bounds__(NT, 1) void k_bmlog(const uint8_t* __restrict__ images, float* __restrict__ pyr,
                                                 const OctJob* __restrict__ jobs, const int32_t* __restrict__ blocks,
                                                 const float* __restrict__ Ht) {
    __shared__ float2 S[BN * HC];   // spectrum
    __shared__ float2 W[BN * HC];   // work buffer
    __shared__ float2 tw[BN];

    const int* blk = blocks + 3 * blockIdx.x;
    const OctJob& job = jobs[blk[0]];
    const int bx = blk[1], by = blk[2];
    const int w = job.w, h = job.h;
    const int x0 = bx * BS - BR, y0 = by * BS - BR;   // image position of block pixel (0, 0)

    if (threadIdx.x < BN) {
        float sn, cs;
        sincospif((float)threadIdx.x / 64.f, &sn, &cs);
        tw[threadIdx.x] = make_float2(cs, -sn);
    }
    // block pixels, rows packed in pairs of columns, in bit-reversed order
    for (int e = threadIdx.x; e < BN * 64; e += NT) {
        const int r = e >> 6, n = e & 63;
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
        S[r * HC + rev6(n)] = make_float2(va, vb);
    }
    __syncthreads();
    rows_fft64<false>(S, tw);
    // split each row's packed transform Z into the spectrum X[0..64] of the
    // real row: E = (Z[k] + conj Z[64-k]) / 2, O = (Z[k] - conj Z[64-k]) / 2i,
    // X[k] = E + w^k O, X[64-k] = conj E - conj(w^k) conj O
    for (int it = threadIdx.x; it < BN * 33; it += NT) {
        const int row = it / 33, k = it - row * 33;
        float2* x = S + row * HC;
        if (k == 0) {
            const float2 z = x[0];
            x[0] = make_float2(z.x + z.y, 0.f);
            x[64] = make_float2(z.x - z.y, 0.f);
        } else {
            const float2 zk = x[k], zm = x[64 - k];
            const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            const float2 O = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            const float2 wk = tw[k];
            const float2 xk = cadd(E, cmul(wk, O));
            const float2 xm = csub(conjf2(E), cmul(conjf2(wk), conjf2(O)));
            x[k] = xk;
            if (k != 32) x[64 - k] = xm;
        }
    }
    __syncthreads();
    // bit-reversed row order for the column transforms
    for (int it = threadIdx.x; it < BN * HC; it += NT) {
        const int r = it / HC, c = it - r * HC, rr = rev7(r);
        if (r < rr) {
            const float2 t = S[r * HC + c];
            S[r * HC + c] = S[rr * HC + c];
            S[rr * HC + c] = t;
        }
    }
    __syncthreads();
    cols_fft128<false>(S, tw);

    const int nout = U8 ? 5 : 4;
    // unnormalised transforms: 128-point columns, then 64-point packed rows
    const float scale = 1.f / (float)(BN * (BN / 2));
    for (int q = 0; q < nout; ++q) {
        const int plane = U8 ? q : q + 1;                     // G_{o,plane}
        const float* H = Ht + (U8 ? (q == 0 ? 0 : 4 + q) : 1 + q) * BN;
        // filtered spectrum, rows bit-reversed for the inverse column FFTs
        for (int it = threadIdx.x; it < BN * HC; it += NT) {
            const int v = it / HC, u = it - v * HC;
            const float g = H[v] * H[u];
            const float2 z = S[it];
            W[rev7(v) * HC + u] = make_float2(z.x * g, z.y * g);
        }
        __syncthreads();
        cols_fft128<true>(W, tw);
        // rebuild each real row's packed transform from its half spectrum:
        // E = (X[k] + conj X[64-k]) / 2, O = (X[k] - conj X[64-k]) conj(w^k) / 2,
        // Z[k] = E + i O (and the same for 64 - k)
        for (int it = threadIdx.x; it < BN * 33; it += NT) {
            const int row = it / 33, k = it - row * 33;
            float2* x = W + row * HC;
            const float2 xk = x[k], xm = x[64 - k];
            const float2 wk = tw[k];
            const float2 E = make_float2(0.5f * (xk.x + xm.x), 0.5f * (xk.y - xm.y));
            const float2 O = cmul(make_float2(0.5f * (xk.x - xm.x), 0.5f * (xk.y + xm.y)), conjf2(wk));
            const float2 zk = make_float2(E.x - O.y, E.y + O.x);   // E + i O
            if (k == 0) {
                x[0] = zk;
            } else if (k == 32) {
                x[32] = zk;
            } else {
                // for 64 - k: E' = conj E, O' = (X[64-k] - conj X[k]) conj(w^(64-k)) / 2,
                // conj(w^(64-k)) = -w^k
                const float2 E2 = conjf2(E);
                const float2 O2 = cmul(make_float2(0.5f * (xm.x - xk.x), 0.5f * (xm.y + xk.y)),
                                       make_float2(-wk.x, -wk.y));
                x[k] = zk;
                x[64 - k] = make_float2(E2.x - O2.y, E2.y + O2.x);
            }
        }
        __syncthreads();
        for (int it = threadIdx.x; it < BN * 64; it += NT) {   // bit-reversed order for the row transforms
            const int r = it >> 6, n = it & 63, nn = rev6(n);
            if (n < nn) {
                const float2 t = W[r * HC + n];
                W[r * HC + n] = W[r * HC + nn];
                W[r * HC + nn] = t;
            }
        }
        __syncthreads();
        rows_fft64<true>(W, tw);
        // central 96 x 96 pixels: element n of row r holds columns 2n, 2n+1
        float* out = pyr + job.plane0 + (int64_t)plane * job.plane_stride;
        const bool down = !U8 ? (q == 3 && job.next0 >= 0) : (q == 4 && job.next0 >= 0);
        for (int it = threadIdx.x; it < BS * (BS / 2); it += NT) {
            const int r = BR + it / (BS / 2), n = BR / 2 + it % (BS / 2);
            const int gy = y0 + r, gx = x0 + 2 * n;
            if (gy >= h || gx >= w) continue;
            const float2 v = W[r * HC + n];
            const float a = v.x * scale, b = v.y * scale;
            float* o = out + (int64_t)gy * job.pitch + gx;
            if (gx + 1 < w) *reinterpret_cast<float2*>(o) = make_float2(a, b);
            else o[0] = a;
            if (down && (gy & 1) == 0) pyr[job.next0 + (int64_t)(gy >> 1) * job.next_pitch + (gx >> 1)] = a;
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
