// ALP keypoint detection on gfx950 (Sec. III-A, Eqs. (2)-(3); Sec. IV-A,
// Algorithm 1 stages A-C).
//
// k_detect: one 256-lane workgroup per 64x16 tile of one (image, octave).
//   The five Gaussian images with a 2-pixel halo are staged in LDS; every
//   lane computes the scale-normalised 5-point Laplacians and the four ALP
//   coefficients of its pixels (tile + 1-pixel halo) into LDS; then per
//   centre pixel: extremal scale, contrast test, strict 8-neighbour test at
//   that scale, one quadratic refinement step.  Survivors are compacted with
//   one wave ballot and one atomic per wave into the image's candidate list.
//   Octaves are launched in order, so each image's list is grouped by octave.
// k_finalize: one workgroup per image.  Stage C (cross-octave duplicates)
//   over adjacent-octave segments, then a bitonic sort in LDS on the 64-bit
//   key (|p| desc, octave, iy, ix) and the top-k copy-out.
#include <algorithm>

#include "cdvs_internal.h"

namespace cdvs {

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

__device__ __forceinline__ int find_det_job(const OctJob* jobs, int njobs, int tile) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0_det <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ float horner(const float4 a, float s) { return fmaf(fmaf(fmaf(a.w, s, a.z), s, a.y), s, a.x); }

// Extremal scale of p(s) = a.x + a.y s + a.z s^2 + a.w s^3 in [lo, hi) where
// |p| has a maximum (p p'' < 0); larger |p| wins, then the smaller s.
__device__ __forceinline__ bool alp_extremum(const float4 a, float lo, float hi, float& s_out, float& p_out,
                                             float& pss_out) {
    const float A = 3.f * a.w, B = 2.f * a.z, C = a.y;
    float r[2];
    int nr = 0;
    if (A == 0.f) {
        if (B != 0.f) r[nr++] = -__fdividef(C, B);
    } else {
        const float disc = B * B - 4.f * A * C;
        if (disc < 0.f) return false;
        const float sq = sqrtf(disc);
        const float q = (B >= 0.f) ? -(B + sq) * 0.5f : -(B - sq) * 0.5f;
        if (q != 0.f) {
            r[nr++] = __fdividef(q, A);
            r[nr++] = __fdividef(C, q);
        } else {
            r[nr++] = 0.f;
        }
    }
    bool found = false;
    float bs = 0.f, bp = 0.f, bpss = 0.f;
    for (int i = 0; i < nr; ++i) {
        const float s = r[i];
        if (!(s >= lo && s < hi)) continue;
        const float p = horner(a, s);
        const float pss = 6.f * a.w * s + 2.f * a.z;
        if (!(p * pss < 0.f)) continue;
        if (!found || fabsf(p) > fabsf(bp) || (fabsf(p) == fabsf(bp) && s < bs)) {
            bs = s;
            bp = p;
            bpss = pss;
            found = true;
        }
    }
    s_out = bs;
    p_out = bp;
    pss_out = bpss;
    return found;
}

constexpr int DTW = kDetTW, DTH = kDetTH;
// staged columns: tx0-4 .. tx0+DTW+3 (16-byte aligned start); rows ty0-2 .. ty0+DTH+1
constexpr int GW = DTW + 8, GH = DTH + 4;
constexpr int GX = 2;  // staged column of image column tx0-2
constexpr int AW = DTW + 2, AH = DTH + 2;

constexpr int DNV4 = kScales * GH * GW / 4;     // float4 chunks of the staged window
constexpr int DNPER4 = (DNV4 + 255) / 256;      // chunks per lane
static_assert(GW % 4 == 0, "staged rows are whole float4 chunks");

// Stage the five planes over the tile plus a clamped halo: rows are clamped
// per chunk; a chunk lying inside the image is one aligned 16-byte load, and
// only chunks crossing the left or right image edge load four clamped
// scalars.  Every load of a lane is issued before its values are needed.
__device__ __forceinline__ void load_tile(const float* __restrict__ pyr, const OctJob& job, int tx0, int ty0,
                                          float4 (&vals)[DNPER4]) {
#pragma unroll
    for (int j = 0; j < DNPER4; ++j) {
        const int t = threadIdx.x + j * 256;
        if (t < DNV4) {
            const int k = t / (GH * GW / 4), rem = t % (GH * GW / 4);
            const int ly = rem / (GW / 4), c4 = rem % (GW / 4);
            const int gy = clampi(ty0 - 2 + ly, 0, job.h - 1);
            const int gx = tx0 - 4 + 4 * c4;
            const float* row = pyr + job.plane0 + (int64_t)k * job.plane_stride + (int64_t)gy * job.pitch;
            if (gx >= 0 && gx + 3 < job.w) {
                vals[j] = *reinterpret_cast<const float4*>(row + gx);
            } else {
                vals[j] = make_float4(row[clampi(gx, 0, job.w - 1)], row[clampi(gx + 1, 0, job.w - 1)],
                                      row[clampi(gx + 2, 0, job.w - 1)], row[clampi(gx + 3, 0, job.w - 1)]);
            }
        }
    }
}

__device__ __forceinline__ void store_tile(float* G, const float4 (&vals)[DNPER4]) {
#pragma unroll
    for (int j = 0; j < DNPER4; ++j) {
        const int t = threadIdx.x + j * 256;
        if (t < DNV4) reinterpret_cast<float4*>(G)[t] = vals[j];
    }
}

// Persistent: the grid (a multiple of 8) is split evenly over the XCDs; each
// workgroup walks its XCD's contiguous tile range with a stride, and the next
// tile's loads are in flight while the current tile is computed.
// Mask gating (optional): an octave-o centre (x, y) is examined only when
// bit o of the mask cell holding (x 2^o, y 2^o) / 4 is set, unless the
// image's active-cell fraction for that octave exceeds gate.fmax (then the
// octave is examined densely).  Tiles without an active centre are skipped
// after staging, and alpha is computed only within one pixel of an active
// centre (every pixel an active centre reads).
__global__ __launch_bounds__(256) void k_detect(const float* __restrict__ pyr, const OctJob* __restrict__ jobs,
                                                int njobs, int ntiles, DetParams dp, GateParams gate,
                                                cdvs_keypoint* __restrict__ cand, int32_t* __restrict__ cand_cnt,
                                                int32_t* __restrict__ flags) {
    __shared__ __align__(16) float G[kScales][GH][GW];
    __shared__ float4 A[AH][AW];
    __shared__ uint8_t act[DTH][DTW];

    const int x = blockIdx.x % kXcds, slot = blockIdx.x / kXcds, nslot = gridDim.x / kXcds;
    const int per = ntiles / kXcds, rem = ntiles % kXcds;
    const int tbase = x * per + min(x, rem), cnt = per + (x < rem ? 1 : 0);
    float4 vals[DNPER4];
    if (slot < cnt) {
        const int tile = tbase + slot;
        const OctJob& job = jobs[find_det_job(jobs, njobs, tile)];
        const int lt = tile - job.tile0_det;
        load_tile(pyr, job, (lt % job.tiles_x_det) * DTW, (lt / job.tiles_x_det) * DTH, vals);
    }
    for (int tj = slot; tj < cnt; tj += nslot) {
        const int tile = tbase + tj;
        const OctJob& job = jobs[find_det_job(jobs, njobs, tile)];
        const int lt = tile - job.tile0_det;
        const int tx0 = (lt % job.tiles_x_det) * DTW;
        const int ty0 = (lt / job.tiles_x_det) * DTH;
        const int w = job.w, h = job.h;

        __syncthreads();  // the previous tile is done with G and A
        store_tile(&G[0][0][0], vals);
        // gating of this tile (uniform across the workgroup)
        bool gated = false;
        if (gate.mask) {
            const CnnImage& cg = gate.cells[job.image];
            const int ncell = cg.H4 * cg.W4;
            gated = (float)gate.active[job.image * kMaxOctaves + job.octave] <= gate.fmax * (float)ncell;
            if (gated) {
                for (int q = threadIdx.x; q < DTH * DTW; q += blockDim.x) {
                    const int gx = tx0 + q % DTW, gy = ty0 + q / DTW;
                    bool on = false;
                    if (gx < w && gy < h) {
                        const int cx = min((gx << job.octave) >> 2, cg.W4 - 1);
                        const int cy = min((gy << job.octave) >> 2, cg.H4 - 1);
                        on = (gate.mask[cg.cell0 + (int64_t)cy * cg.W4 + cx] >> job.octave) & 1;
                    }
                    act[q / DTW][q % DTW] = on;
                }
            }
        }
        // (the barrier inside __syncthreads_or publishes G and act)
        if (__syncthreads_or(gated && threadIdx.x == 0)) {
            // any active centre in the tile?
            bool mine = false;
            for (int q = threadIdx.x; q < DTH * DTW; q += blockDim.x) mine |= act[q / DTW][q % DTW] != 0;
            if (!__syncthreads_or(mine)) {
                if (tj + nslot < cnt) {
                    const int tn = tbase + tj + nslot;
                    const OctJob& jn = jobs[find_det_job(jobs, njobs, tn)];
                    const int ltn = tn - jn.tile0_det;
                    load_tile(pyr, jn, (ltn % jn.tiles_x_det) * DTW, (ltn / jn.tiles_x_det) * DTH, vals);
                }
                continue;
            }
        }
        if (tj + nslot < cnt) {
            const int tn = tbase + tj + nslot;
            const OctJob& jn = jobs[find_det_job(jobs, njobs, tn)];
            const int ltn = tn - jn.tile0_det;
            load_tile(pyr, jn, (ltn % jn.tiles_x_det) * DTW, (ltn / jn.tiles_x_det) * DTH, vals);
        }

        for (int t = threadIdx.x; t < AH * AW; t += blockDim.x) {
            const int ay = t / AW, ax = t % AW;
            const int ly = ay + 1, lx = ax + 1 + GX;
            if (gated) {
                // alpha at (ay, ax) is read only by centres (ay-1+dy, ax-1+dx)
                bool need = false;
                for (int dy = -2; dy <= 0; ++dy)
                    for (int dx = -2; dx <= 0; ++dx) {
                        const int cy = ay + dy, cx = ax + dx;
                        if (cy >= 0 && cy < DTH && cx >= 0 && cx < DTW) need |= act[cy][cx] != 0;
                    }
                if (!need) continue;
            }
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
            for (int k = 0; k < kScales; ++k) {
                const float c = G[k][ly][lx];
                float s = G[k][ly - 1][lx] + G[k][ly + 1][lx];
                s = s + G[k][ly][lx - 1];
                s = s + G[k][ly][lx + 1];
                s = s - 4.f * c;
                const float L = dp.sig2[k] * s;
                a0 = fmaf(dp.beta[k][0], L, a0);
                a1 = fmaf(dp.beta[k][1], L, a1);
                a2 = fmaf(dp.beta[k][2], L, a2);
                a3 = fmaf(dp.beta[k][3], L, a3);
            }
            A[ay][ax] = make_float4(a0, a1, a2, a3);
        }
        __syncthreads();

        const int lane = threadIdx.x & 63;
        const float scale = (float)(1 << job.octave);
        for (int it = 0; it < DTW * DTH / 256; ++it) {
            const int q = threadIdx.x + it * 256;
            const int cy = q / DTW, cx = q % DTW;
            const int gx = tx0 + cx, gy = ty0 + cy;
            bool keep = false;
            float s = 0.f, p = 0.f, pss = 0.f, ox = 0.f, oy = 0.f, pr = 0.f, rho = 0.f;
            if (gx >= dp.border && gx <= w - 1 - dp.border && gy >= dp.border && gy <= h - 1 - dp.border &&
                (!gated || act[cy][cx])) {
                const float4 a = A[cy + 1][cx + 1];
                if (alp_extremum(a, dp.lo, dp.hi, s, p, pss) && fabsf(p) >= dp.contrast) {
                    float v[9];
                    bool ext = true;
#pragma unroll
                    for (int j = -1; j <= 1; ++j)
#pragma unroll
                        for (int i = -1; i <= 1; ++i) {
                            if (i == 0 && j == 0) {
                                v[4] = p;
                                continue;
                            }
                            const float qv = horner(A[cy + 1 + j][cx + 1 + i], s);
                            v[(j + 1) * 3 + (i + 1)] = qv;
                            ext = ext && (p > 0.f ? (qv < p) : (qv > p));
                        }
                    if (ext) {
                        const float c = v[4];
                        const float gxd = (v[5] - v[3]) * 0.5f;
                        const float gyd = (v[7] - v[1]) * 0.5f;
                        const float hxx = v[5] - 2.f * c + v[3];
                        const float hyy = v[7] - 2.f * c + v[1];
                        const float hxy = (v[8] - v[6] - v[2] + v[0]) * 0.25f;
                        const float det = hxx * hyy - hxy * hxy;
                        if (det > 0.f) {
                            const float tr = hxx + hyy;
                            const float ratio = __fdividef(tr * tr, det);
                            if (ratio < dp.edge_lim) {
                                const float rdet = 1.f / det;
                                const float dx = -(hyy * gxd - hxy * gyd) * rdet;
                                const float dy = -(hxx * gyd - hxy * gxd) * rdet;
                                if (!(fabsf(dx) > dp.max_off || fabsf(dy) > dp.max_off)) {
                                    ox = dx;
                                    oy = dy;
                                    pr = c + (gxd * dx + gyd * dy) * 0.5f;
                                    rho = ratio;
                                    keep = true;
                                }
                            }
                        }
                    }
                }
            }
            const uint64_t m = __ballot(keep);
            if (m) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&cand_cnt[job.image], __popcll(m));
                base = __shfl(base, leader);
                if (keep) {
                    const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
                    if (slot < dp.cand_cap) {
                        cdvs_keypoint r;
                        r.x = ((float)gx + ox) * scale;
                        r.y = ((float)gy + oy) * scale;
                        r.sigma = s * scale;
                        r.p = pr;
                        r.theta = 0.f;
                        r.rho = rho;
                        r.p_ss = pss;
                        r.peak = 0.f;
                        r.image = job.image;
                        r.octave = job.octave;
                        r.ix = gx;
                        r.iy = gy;
                        cand[(int64_t)job.image * dp.cand_cap + slot] = r;
                    } else {
                        atomicOr(flags, kFlagCandOverflow);
                    }
                }
            }
        }
    }
}

__global__ void k_clear(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

constexpr int FIN_THREADS = 1024;
constexpr int FIN_PER = kCandCap / FIN_THREADS;  // candidates per thread

// Stage C + canonical sort + top-k for one image per workgroup.  The
// candidates' (x, y, sigma, p) are staged in LDS for the pair loop; the same
// LDS then holds the sort keys.
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const cdvs_keypoint* __restrict__ cand,
                                                          const int32_t* __restrict__ cand_cnt, int cand_cap,
                                                          float ratio_lim, int topk, int kp_cap,
                                                          cdvs_keypoint* __restrict__ kp,
                                                          int32_t* __restrict__ count) {
    // records: kCandCap float4 = 128 KB; keys + indices reuse the same bytes
    __shared__ float4 rec[kCandCap];
    __shared__ int seg[kMaxOctaves + 2];
    __shared__ int n_alive;
    unsigned long long* key = reinterpret_cast<unsigned long long*>(rec);
    unsigned short* idx = reinterpret_cast<unsigned short*>(key + kCandCap);

    const int img = blockIdx.x;
    const cdvs_keypoint* c = cand + (int64_t)img * cand_cap;
    const int n = min(cand_cnt[img], cand_cap);
    const int tid = threadIdx.x;

    if (tid < kMaxOctaves + 2) seg[tid] = n;
    if (tid == 0) n_alive = 0;
    __syncthreads();
    int oct[FIN_PER];
#pragma unroll
    for (int j = 0; j < FIN_PER; ++j) {
        const int i = tid + j * FIN_THREADS;
        oct[j] = -1;
        if (i < n) {
            const cdvs_keypoint a = c[i];
            rec[i] = make_float4(a.x, a.y, a.sigma, a.p);
            oct[j] = a.octave;
            // seg[o] = first index whose octave >= o (the list is grouped by octave)
            const int prev = (i == 0) ? -1 : c[i - 1].octave;
            for (int o = prev + 1; o <= a.octave; ++o) seg[o] = i;
        }
    }
    __syncthreads();

    unsigned long long kk[FIN_PER];
    int local_alive = 0;
#pragma unroll
    for (int j = 0; j < FIN_PER; ++j) {
        const int i = tid + j * FIN_THREADS;
        kk[j] = ~0ull;
        if (i < n) {
            const float4 a = rec[i];
            const int ao = oct[j];
            const float aa = fabsf(a.w);
            bool alive = true;
            for (int d = -1; d <= 1 && alive; d += 2) {
                const int o2 = ao + d;
                if (o2 < 0 || o2 >= kMaxOctaves) continue;
                const float lim = (float)(1 << max(ao, o2));
                const float lim2 = lim * lim;
                for (int jj = seg[o2]; jj < seg[o2 + 1]; ++jj) {
                    const float4 b = rec[jj];
                    if ((a.w > 0.f) != (b.w > 0.f)) continue;
                    const float dx = a.x - b.x, dy = a.y - b.y;
                    if (!(dx * dx + dy * dy <= lim2)) continue;
                    const float shi = fmaxf(a.z, b.z), slo = fminf(a.z, b.z);
                    if (!(shi <= ratio_lim * slo)) continue;
                    const float ab = fabsf(b.w);
                    if (ab > aa || (ab == aa && o2 < ao)) {
                        alive = false;
                        break;
                    }
                }
            }
            if (alive) {
                ++local_alive;
                const cdvs_keypoint& r = c[i];
                kk[j] = ((unsigned long long)(~__float_as_uint(aa)) << 32) |
                        ((unsigned long long)ao << 28) | ((unsigned long long)r.iy << 14) |
                        (unsigned long long)r.ix;
            }
        }
    }
    if (local_alive) atomicAdd(&n_alive, local_alive);
    int npow = 1;
    while (npow < n) npow <<= 1;
    __syncthreads();  // every lane is done reading rec[] before keys overwrite it
#pragma unroll
    for (int j = 0; j < FIN_PER; ++j) {
        const int i = tid + j * FIN_THREADS;
        if (i < npow) {
            key[i] = kk[j];
            idx[i] = (unsigned short)i;
        }
    }
    __syncthreads();

    // bitonic sort, ascending
    for (int size = 2; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < npow / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const unsigned long long kl = key[lo], kh = key[hi];
                if ((kl > kh) == asc) {
                    key[lo] = kh;
                    key[hi] = kl;
                    const unsigned short il = idx[lo];
                    idx[lo] = idx[hi];
                    idx[hi] = il;
                }
            }
            __syncthreads();
        }
    }

    const int limit = min(topk > 0 ? topk : kp_cap, kp_cap);
    const int m = min(n_alive, limit);
    for (int r = tid; r < m; r += blockDim.x) kp[(int64_t)img * kp_cap + r] = c[idx[r]];
    if (tid == 0) count[img] = m;
}

}  // namespace

hipError_t launch_clear(int32_t* p, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_detect(const float* pyr, const OctJob* jobs, int njobs, int ntiles, int grid, const DetParams& dp,
                         const GateParams& gate, cdvs_keypoint* cand, int32_t* cand_cnt, int32_t* flags,
                         hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    // a multiple of the XCD count, no larger than needed
    int g = std::min(grid, (ntiles + kXcds - 1) / kXcds * kXcds);
    g = std::max(kXcds, g / kXcds * kXcds);
    hipLaunchKernelGGL(k_detect, dim3(g), dim3(256), 0, stream, pyr, jobs, njobs, ntiles, dp, gate, cand, cand_cnt,
                       flags);
    return hipGetLastError();
}

hipError_t launch_finalize(const cdvs_keypoint* cand, const int32_t* cand_cnt, int n_images, int cand_cap,
                           float dedup_ratio, int topk, int kp_cap, cdvs_keypoint* kp, int32_t* count,
                           hipStream_t stream) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(n_images), dim3(FIN_THREADS), 0, stream, cand, cand_cnt, cand_cap,
                       dedup_ratio, topk, kp_cap, kp, count);
    return hipGetLastError();
}

}  // namespace cdvs
