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
//   One persistent launch per octave covers that octave of every image.
// k_finalize: one workgroup per image.  Stage C (cross-octave duplicates)
//   over adjacent-octave segments, then a bitonic sort in LDS on the 64-bit
//   key (|p| desc, octave, iy, ix) and the top-k copy-out.
#include <algorithm>

#include "cdvs_internal.h"

namespace cdvs {

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

__device__ __forceinline__ float horner(const float4 a, float s) { return fmaf(fmaf(fmaf(a.w, s, a.z), s, a.y), s, a.x); }

// Extremal scale of p(s) = a.x + a.y s + a.z s^2 + a.w s^3 in [lo, hi) where
// |p| has a maximum (p p'' < 0); larger |p| wins, then the smaller s.
__device__ __forceinline__ bool alp_extremum(const float4 a, float lo, float hi, float& s_out, float& p_out,
                                             float& pss_out) {
    const float A = 3.f * a.w, B = 2.f * a.z, C = a.y;
    float r[2];
    int nr = 0;
    // quotients by the hardware reciprocal (1 ulp) and a multiply: a plain
    // division is a full IEEE sequence on this target, several times longer
    if (A == 0.f) {
        if (B != 0.f) r[nr++] = -(C * __builtin_amdgcn_rcpf(B));
    } else {
        const float disc = B * B - 4.f * A * C;
        if (disc < 0.f) return false;
        const float sq = __builtin_amdgcn_sqrtf(disc);   // hardware square root (1 ulp)
        const float q = (B >= 0.f) ? -(B + sq) * 0.5f : -(B - sq) * 0.5f;
        if (q != 0.f) {
            r[nr++] = q * __builtin_amdgcn_rcpf(A);
            r[nr++] = C * __builtin_amdgcn_rcpf(q);
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
// After the coefficients are computed the staging buffer holds the list of
// contrast-passing centres (16 B each, at most one per centre).
static_assert(kScales * GH * GW >= 4 * DTW * DTH, "the staging buffer holds the list of every centre");

// Stage the five planes over the tile plus a clamped halo: rows are clamped
// per chunk; a chunk lying inside the image is one aligned 16-byte load, and
// only chunks crossing the left or right image edge load four clamped
// scalars.  Every load of a lane is issued before its values are needed.
__device__ __forceinline__ void load_tile(const float* __restrict__ pyr, const DetTile& job, float4 (&vals)[DNPER4]) {
    const int tx0 = job.tx0, ty0 = job.ty0;
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

// Scale-normalised 5-point Laplacians of the five planes at staged pixel
// (ly, lx), folded into the four ALP coefficients (Eqs. (2)-(3)).
// 5-point Laplacian sum (up + down + left + right - 4 centre), in one fixed
// order of operations shared by both detection kernels.
__device__ __forceinline__ float lap5(float c, float up, float dn, float lf, float rt) {
    float s = up + dn;
    s = s + lf;
    s = s + rt;
    s = s - 4.f * c;
    return s;
}

// Adds scale k's normalised Laplacian to the ALP coefficients.
__device__ __forceinline__ void alpha_acc(float4& a, float lap, int k, const DetParams& dp) {
    const float L = dp.sig2[k] * lap;
    a.x = fmaf(dp.beta[k][0], L, a.x);
    a.y = fmaf(dp.beta[k][1], L, a.y);
    a.z = fmaf(dp.beta[k][2], L, a.z);
    a.w = fmaf(dp.beta[k][3], L, a.w);
}

__device__ __forceinline__ float4 alpha_at(const float (&G)[kScales][GH][GW], int ly, int lx, const DetParams& dp) {
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < kScales; ++k)
        alpha_acc(a, lap5(G[k][ly][lx], G[k][ly - 1][lx], G[k][ly + 1][lx], G[k][ly][lx - 1], G[k][ly][lx + 1]), k,
                  dp);
    return a;
}

struct Cand {
    float s, p, pss, ox, oy, pr, rho;
};

// Tile centre (cy, cx), first half: extremal scale and contrast.
__device__ __forceinline__ bool centre_extremum(const float4 (&A)[AH][AW], int cy, int cx, const DetParams& dp,
                                                float& s, float& p, float& pss) {
    return alp_extremum(A[cy + 1][cx + 1], dp.lo, dp.hi, s, p, pss) && fabsf(p) >= dp.contrast;
}

// Strict extremum of the centre value p = v[4] against the eight
// neighbours' cubics v[] evaluated at the centre's scale (Algorithm 1 stage A).
__device__ __forceinline__ bool strict_extremum(const float (&v)[9], float p) {
    bool ext = true;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (i != 4) ext = ext && (p > 0.f ? (v[i] < p) : (v[i] > p));
    return ext;
}

// One quadratic refinement step on the 3x3 values v[] (row-major, centre
// v[4] = p): offset, edge test and interpolated response (Algorithm 1 stage B).
__device__ __forceinline__ bool refine_v(const float (&v)[9], float s, float p, float pss, const DetParams& dp,
                                         Cand& o) {
    const float c = v[4];
    const float gxd = (v[5] - v[3]) * 0.5f;
    const float gyd = (v[7] - v[1]) * 0.5f;
    const float hxx = v[5] - 2.f * c + v[3];
    const float hyy = v[7] - 2.f * c + v[1];
    const float hxy = (v[8] - v[6] - v[2] + v[0]) * 0.25f;
    const float det = hxx * hyy - hxy * hxy;
    if (!(det > 0.f)) return false;
    const float tr = hxx + hyy;
    const float ratio = __fdividef(tr * tr, det);
    if (!(ratio < dp.edge_lim)) return false;
    const float rdet = 1.f / det;
    const float dx = -(hyy * gxd - hxy * gyd) * rdet;
    const float dy = -(hxx * gyd - hxy * gxd) * rdet;
    if (fabsf(dx) > dp.max_off || fabsf(dy) > dp.max_off) return false;
    o.s = s;
    o.p = p;
    o.pss = pss;
    o.ox = dx;
    o.oy = dy;
    o.pr = c + (gxd * dx + gyd * dy) * 0.5f;
    o.rho = ratio;
    return true;
}

// Second half for a staged tile: strict 8-neighbour test at the centre's
// scale and one quadratic refinement step (Algorithm 1 stages A-B).
__device__ __forceinline__ bool centre_refine(const float4 (&A)[AH][AW], int cy, int cx, float s, float p, float pss,
                                              const DetParams& dp, Cand& o) {
    float v[9];
#pragma unroll
    for (int j = -1; j <= 1; ++j)
#pragma unroll
        for (int i = -1; i <= 1; ++i) v[(j + 1) * 3 + (i + 1)] = (i == 0 && j == 0) ? p : horner(A[cy + 1 + j][cx + 1 + i], s);
    return strict_extremum(v, p) && refine_v(v, s, p, pss, dp, o);
}

// Appends (s, p, pss, centre index) of the lanes with `pass` to an LDS list
// (one ballot and one LDS atomic per wave).  Every lane of the wave calls it.
__device__ __forceinline__ void push_centre(bool pass, float s, float p, float pss, int q, float4* list, int* count) {
    const int lane = threadIdx.x & 63;
    const uint64_t m = __ballot(pass);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, leader);
    if (pass) list[base + __popcll(m & ((1ull << lane) - 1ull))] = make_float4(s, p, pss, __int_as_float(q));
}

// Wave-level compaction of survivors into the image's candidate list: one
// ballot and one atomic per wave.  Every lane of the wave must call it.
__device__ __forceinline__ void emit(bool keep, const Cand& c, int gx, int gy, const DetTile& job, const DetParams& dp,
                                     cdvs_keypoint* __restrict__ cand, int32_t* __restrict__ cand_cnt,
                                     int32_t* __restrict__ flags) {
    const int lane = threadIdx.x & 63;
    const uint64_t m = __ballot(keep);
    if (!m) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&cand_cnt[job.image], __popcll(m));
    base = __shfl(base, leader);
    if (!keep) return;
    const int slot = base + __popcll(m & ((1ull << lane) - 1ull));
    if (slot >= job.cand_cap) {
        atomicOr(flags, kFlagCandOverflow);
        return;
    }
    const float scale = (float)(1 << job.octave);
    cdvs_keypoint r;
    r.x = ((float)gx + c.ox) * scale;
    r.y = ((float)gy + c.oy) * scale;
    r.sigma = c.s * scale;
    r.p = c.pr;
    r.theta = 0.f;
    r.rho = c.rho;
    r.p_ss = c.pss;
    r.peak = 0.f;
    r.image = job.image;
    r.octave = job.octave;
    r.ix = gx;
    r.iy = gy;
    cand[(int64_t)job.cand_blk * kCandBlock + slot] = r;
}

// Second phase over the LDS list of contrast-passing centres: dense lanes
// for the 3x3 test and refinement, survivors appended to the candidates.
__device__ __forceinline__ void refine_list(const float4 (&A)[AH][AW], const float4* list, int n, const DetTile& job,
                                           const DetParams& dp, cdvs_keypoint* __restrict__ cand,
                                           int32_t* __restrict__ cand_cnt, int32_t* __restrict__ flags) {
    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x;
        Cand c{};
        bool keep = false;
        int gx = 0, gy = 0;
        if (i < n) {
            const float4 r = list[i];
            const int q = __float_as_int(r.w);
            const int cy = q / DTW, cx = q % DTW;
            gx = job.tx0 + cx;
            gy = job.ty0 + cy;
            keep = centre_refine(A, cy, cx, r.x, r.y, r.z, dp, c);
        }
        emit(keep, c, gx, gy, job, dp, cand, cand_cnt, flags);
    }
}

// Tile records are fetched with vector loads, lane i holding dword i (the
// wait for a scalar load would come at the next LDS access, since both are
// counted together); as_uniform() moves the fields to scalar registers once
// the record has arrived.
typedef int RawTile;

__device__ __forceinline__ RawTile fetch_tile(const DetTile* __restrict__ tiles, int idx) {
    const int lane = threadIdx.x & 63;
    constexpr int kWords = (int)sizeof(DetTile) / 4;
    return reinterpret_cast<const int*>(tiles + idx)[min(lane, kWords - 1)];
}

__device__ __forceinline__ DetTile as_uniform(RawTile r) {
    DetTile t;
    t.plane0 = (int64_t)(uint32_t)__builtin_amdgcn_readlane(r, 0) | ((int64_t)__builtin_amdgcn_readlane(r, 1) << 32);
    t.plane_stride = __builtin_amdgcn_readlane(r, 2);
    t.pitch = __builtin_amdgcn_readlane(r, 3);
    t.w = __builtin_amdgcn_readlane(r, 4);
    t.h = __builtin_amdgcn_readlane(r, 5);
    t.tx0 = __builtin_amdgcn_readlane(r, 6);
    t.ty0 = __builtin_amdgcn_readlane(r, 7);
    t.image = __builtin_amdgcn_readlane(r, 8);
    t.octave = __builtin_amdgcn_readlane(r, 9);
    t.cand_cap = __builtin_amdgcn_readlane(r, 10);
    t.cand_blk = __builtin_amdgcn_readlane(r, 11);
    return t;
}

// Persistent: the grid (a multiple of 8) is split evenly over the XCDs; each
// workgroup walks its XCD's contiguous tile range with a stride, and the next
// tile's loads are in flight while the current tile is computed.
// The refinement of a tile's contrast-passing centres (which ends in global
// atomics whose results are awaited) runs at the start of the next
// iteration, before that iteration issues its prefetch: a wait on a global
// atomic also waits for every vector load issued before it, so this way the
// prefetched planes are in flight during the coefficients and extremal
// scales, and the atomics only ever wait for loads about to be consumed.
__global__ __launch_bounds__(256) void k_detect(const float* __restrict__ pyr, const DetTile* __restrict__ tiles,
                                                int ntiles, DetParams dp, cdvs_keypoint* __restrict__ cand,
                                                int32_t* __restrict__ cand_cnt, int32_t* __restrict__ flags) {
    __shared__ __align__(16) float G[kScales][GH][GW];
    __shared__ float4 A[AH][AW];
    __shared__ int nlist;

    const int x = blockIdx.x % kXcds, slot = blockIdx.x / kXcds, nslot = gridDim.x / kXcds;
    const int per = ntiles / kXcds, rem = ntiles % kXcds;
    const int tbase = x * per + min(x, rem), cnt = per + (x < rem ? 1 : 0);
    if (slot >= cnt) return;   // uniform over the workgroup
    float4* list = reinterpret_cast<float4*>(&G[0][0][0]);   // contrast-passing centres, after the coefficients
    float4 vals[DNPER4];
    DetTile cur = as_uniform(fetch_tile(tiles, tbase + slot));
    DetTile prev = cur;
    load_tile(pyr, cur, vals);
    RawTile rn = fetch_tile(tiles, tbase + min(slot + nslot, cnt - 1));
    for (int tj = slot; tj < cnt; tj += nslot) {
        // the record two tiles ahead is fetched a whole tile before it is needed
        const RawTile rnn = fetch_tile(tiles, tbase + min(tj + 2 * nslot, cnt - 1));
        const DetTile nxt = as_uniform(rn);
        __syncthreads();  // the previous tile's list and coefficients are complete
        if (tj != slot) refine_list(A, list, nlist, prev, dp, cand, cand_cnt, flags);
        __syncthreads();  // the previous tile is done with G, A and the list
        store_tile(&G[0][0][0], vals);
        if (threadIdx.x == 0) nlist = 0;
        __syncthreads();
        if (tj + nslot < cnt) load_tile(pyr, nxt, vals);
        for (int t = threadIdx.x; t < AH * AW; t += blockDim.x) {
            const int ay = t / AW, ax = t % AW;
            A[ay][ax] = alpha_at(G, ay + 1, ax + 1 + GX, dp);
        }
        __syncthreads();
        for (int it = 0; it < DTW * DTH / 256; ++it) {
            const int q = threadIdx.x + it * 256;
            const int cy = q / DTW, cx = q % DTW;
            const int gx = cur.tx0 + cx, gy = cur.ty0 + cy;
            float cs = 0.f, cp = 0.f, cpss = 0.f;
            const bool pass = gx >= dp.border && gx <= cur.w - 1 - dp.border && gy >= dp.border &&
                              gy <= cur.h - 1 - dp.border && centre_extremum(A, cy, cx, dp, cs, cp, cpss);
            push_centre(pass, cs, cp, cpss, q, list, &nlist);
        }
        prev = cur;
        cur = nxt;
        rn = rnn;
    }
    __syncthreads();
    refine_list(A, list, nlist, prev, dp, cand, cand_cnt, flags);
}

// ---------------------------------------------------------------------------
// k_detect_strip: the ungated detection, one wave per strip of kStripW
// centre columns x kStripH centre rows of one (image, octave) inside the
// detection border; lane l holds image column x0 - 2 + l (lanes 0, 1, 62
// and 63 are halo).  The wave walks down its strip one row at a time with
// no LDS staging and no barriers: each row's five plane values arrive by one
// coalesced dword load per plane, issued a chunk of rows ahead; the
// Laplacians take their horizontal neighbours from the adjacent lanes (DPP
// wave shifts) and their vertical ones from the previous two rows held in
// registers, and the ALP coefficients of the last three rows stay in
// registers for the centre tests.  For the strict 3x3 test each lane
// evaluates its own column's cubics at its neighbours' scales and hands the
// values over, so no lane needs another lane's coefficients.  Centres that
// pass are queued in the wave's LDS list with their 3x3 values and refined
// in passes of up to 64 once more than 36 are waiting (dense lanes; one
// global atomic per pass).
constexpr int kStripW = kDetStripW;
constexpr int kStripH = kDetStripH;
constexpr int kQCap = 96;              // flushed above 36, and one row adds at most 60
constexpr int kQFlush = kQCap - 60;
constexpr int kQFields = 12;           // the eight neighbour values, s, p, pss, (x | y << 16)

__device__ __forceinline__ float lane_from_left(float v) {   // lane l gets lane l-1's value (lane 0: 0)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_from_right(float v) {  // lane l gets lane l+1's value (lane 63: 0)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

struct StripRow {
    float g[kScales];
};

// Plane row y (clamped to the image) of this lane's column.
__device__ __forceinline__ void load_row(const float* __restrict__ col, const DetTile& job, int y, StripRow& r) {
    const float* p = col + (int64_t)clampi(y, 0, job.h - 1) * job.pitch;
#pragma unroll
    for (int k = 0; k < kScales; ++k) r.g[k] = p[(int64_t)k * job.plane_stride];
}

// ALP coefficients of the middle row from three consecutive rows.
__device__ __forceinline__ float4 strip_alpha(const StripRow& u, const StripRow& m, const StripRow& d,
                                              const DetParams& dp) {
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < kScales; ++k)
        alpha_acc(a, lap5(m.g[k], u.g[k], d.g[k], lane_from_left(m.g[k]), lane_from_right(m.g[k])), k, dp);
    return a;
}

// Refines queued centres base .. base+n-1 (n <= 64) of this wave and
// appends the survivors to the image's candidates.  Every lane of the wave
// calls it.
__device__ __forceinline__ void strip_flush(float (*q)[kQCap], int base, int n, const DetTile& job,
                                            const DetParams& dp, cdvs_keypoint* __restrict__ cand,
                                            int32_t* __restrict__ cand_cnt, int32_t* __restrict__ flags) {
    const int lane = threadIdx.x & 63;
    Cand c{};
    bool keep = false;
    int gx = 0, gy = 0;
    if (lane < n) {
        const int e = base + lane;
        float v[9];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = q[i][e];
        v[4] = q[9][e];   // the centre: p
#pragma unroll
        for (int i = 5; i < 9; ++i) v[i] = q[i - 1][e];
        const int xy = __float_as_int(q[11][e]);
        gx = xy & 0xffff;
        gy = xy >> 16;
        keep = refine_v(v, q[8][e], q[9][e], q[10][e], dp, c);
    }
    emit(keep, c, gx, gy, job, dp, cand, cand_cnt, flags);
}

// Refines everything queued (in passes of 64) and empties the queue.
__device__ __forceinline__ void strip_drain(float (*q)[kQCap], int& qn, const DetTile& job, const DetParams& dp,
                                            cdvs_keypoint* __restrict__ cand, int32_t* __restrict__ cand_cnt,
                                            int32_t* __restrict__ flags) {
    for (int base = 0; base < qn; base += 64) strip_flush(q, base, min(64, qn - base), job, dp, cand, cand_cnt, flags);
    qn = 0;
}

// Centre tests of one row y from the coefficients of rows y-1, y, y+1;
// strict extrema are queued (qn: the wave's queue length, uniform).
__device__ __forceinline__ void strip_centres(const float4& aU, const float4& aM, const float4& aD, bool col_ok, int gx,
                                              int y, float (*q)[kQCap], int& qn, const DetTile& job,
                                              const DetParams& dp, cdvs_keypoint* __restrict__ cand,
                                              int32_t* __restrict__ cand_cnt, int32_t* __restrict__ flags) {
    float s = 0.f, p = 0.f, pss = 0.f;
    const bool pass = col_ok && alp_extremum(aM, dp.lo, dp.hi, s, p, pss) && fabsf(p) >= dp.contrast;
    if (!__ballot(pass)) return;   // uniform over the wave
    // this lane's column at the scale of the centre to its right (for which
    // it is the left column) and of the centre to its left
    const float s_r = lane_from_right(s), s_l = lane_from_left(s);
    const float l0 = horner(aU, s_r), l1 = horner(aM, s_r), l2 = horner(aD, s_r);
    const float r0 = horner(aU, s_l), r1 = horner(aM, s_l), r2 = horner(aD, s_l);
    float v[9];
    v[0] = lane_from_left(l0);
    v[3] = lane_from_left(l1);
    v[6] = lane_from_left(l2);
    v[2] = lane_from_right(r0);
    v[5] = lane_from_right(r1);
    v[8] = lane_from_right(r2);
    v[1] = horner(aU, s);
    v[4] = p;
    v[7] = horner(aD, s);
    const bool keep = pass && strict_extremum(v, p);
    const uint64_t m = __ballot(keep);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    if (keep) {
        const int i = qn + __popcll(m & ((1ull << lane) - 1ull));
#pragma unroll
        for (int f = 0; f < 4; ++f) q[f][i] = v[f];
#pragma unroll
        for (int f = 5; f < 9; ++f) q[f - 1][i] = v[f];
        q[8][i] = s;
        q[9][i] = p;
        q[10][i] = pss;
        q[11][i] = __int_as_float(gx | (y << 16));
    }
    qn += __popcll(m);
    if (qn > kQFlush) strip_drain(q, qn, job, dp, cand, cand_cnt, flags);
}

__global__ __launch_bounds__(256) void k_detect_strip(const float* __restrict__ pyr, const DetTile* __restrict__ strips,
                                                      int nstrips, DetParams dp, cdvs_keypoint* __restrict__ cand,
                                                      int32_t* __restrict__ cand_cnt, int32_t* __restrict__ flags) {
    __shared__ float queue[4][kQFields][kQCap];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sidx = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * 4 + wave);
    if (sidx >= nstrips) return;   // uniform over the wave; there are no barriers
    float (*q)[kQCap] = queue[wave];
    const DetTile job = strips[sidx];
    const int x0 = job.tx0, y0 = job.ty0;
    const int xend = min(x0 + kStripW, job.w - dp.border), yend = min(y0 + kStripH, job.h - dp.border);
    const int gx = x0 - 2 + lane;
    const bool col_ok = lane >= 2 && gx < xend;
    const float* col = pyr + job.plane0 + clampi(gx, 0, job.w - 1);
    // Plane rows live in a ring of kRing slots, row y in slot (y - y0 + 2) %
    // kRing, and coefficient rows in a ring of three, row y in slot
    // (y - y0 + 1) % 3.  Centre row y computes the coefficients of row y+1,
    // which frees plane row y's slot for row y + kRing, loaded right away and
    // first needed four rows later.  Loads past the strip's last plane row
    // re-read that row (clamped; every load is unconditional, so the waits
    // for them are exact).
    constexpr int kRing = 6;
    const int last = yend + 1;
    StripRow g[kRing], t0, t1;
    load_row(col, job, y0 - 2, t0);
    load_row(col, job, y0 - 1, t1);
#pragma unroll
    for (int r = 2; r < kRing + 2; ++r) load_row(col, job, min(y0 - 2 + r, last), g[r % kRing]);
    float4 a[3];
    a[0] = strip_alpha(t0, t1, g[2], dp);     // row y0-1
    a[1] = strip_alpha(t1, g[2], g[3], dp);   // row y0
    int qn = 0;
    for (int y = y0; y < yend; y += kRing) {
#pragma unroll
        for (int r = 0; r < kRing; ++r) {
            a[(r + 2) % 3] = strip_alpha(g[(r + 2) % kRing], g[(r + 3) % kRing], g[(r + 4) % kRing], dp);
            load_row(col, job, min(y + r + kRing, last), g[(r + 2) % kRing]);
            if (y + r < yend)   // uniform over the wave
                strip_centres(a[r % 3], a[(r + 1) % 3], a[(r + 2) % 3], col_ok, gx, y + r, q, qn, job, dp, cand,
                              cand_cnt, flags);
        }
    }
    strip_drain(q, qn, job, dp, cand, cand_cnt, flags);
}

// Gating pre-pass, one wave per detection tile (all octaves in one
// launch): the tile's active-centre row masks (bit cx of row cy) and its
// state.  An octave-o centre (x, y) is active when it lies inside the
// detection border and bit o of the mask cell holding (x 2^o, y 2^o) / 4 is
// set; when the image's active-cell fraction for that octave exceeds
// gate.fmax the whole octave is dense (every border-valid centre active).
__global__ __launch_bounds__(256) void k_gate_rows(const DetTile* __restrict__ tiles, int ntiles, DetParams dp,
                                                   GateParams gate, uint64_t* __restrict__ rows_out,
                                                   int32_t* __restrict__ state_out) {
    // one wave per tile, lane = tile column
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (tile >= ntiles) return;   // uniform over the wave
    const DetTile job = tiles[tile];
    const CnnImage& cg = gate.cells[job.image];
    const bool dense = (float)gate.active[job.image * kMaxOctaves + job.octave] > gate.fmax * (float)(cg.H4 * cg.W4);
    const int gx = job.tx0 + lane;
    const int cx = min((gx << job.octave) >> 2, cg.W4 - 1);
    const bool colok = gx >= dp.border && gx <= job.w - 1 - dp.border;
    bool any = false;
    for (int cy = 0; cy < DTH; ++cy) {
        const int gy = job.ty0 + cy;
        bool on = colok && gy >= dp.border && gy <= job.h - 1 - dp.border;
        if (on && !dense) {
            const int cyc = min((gy << job.octave) >> 2, cg.H4 - 1);
            on = (gate.mask[cg.cell0 + (int64_t)cyc * cg.W4 + cx] >> job.octave) & 1;
        }
        const uint64_t m = __ballot(on);
        if (lane == cy) rows_out[(int64_t)tile * DTH + cy] = m;
        any |= m != 0;
    }
    if (lane == 0) state_out[tile] = !any ? kTileSkip : (dense ? kTileDense : kTileSparse);
}

// Exclusive prefix of the values held by the lanes of a wave.
__device__ __forceinline__ int wave_excl_scan(int v) {
    const int lane = threadIdx.x & 63;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    return x - v;
}

// A tile's gating state and row masks, fetched with vector loads like the
// tile record (lanes 0..15 each hold one row).
struct RawGate {
    int state;
    uint64_t row;
};

__device__ __forceinline__ RawGate fetch_gate(const GateParams& gate, int idx) {
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    const int lane = threadIdx.x & 63;
    RawGate r;
    r.state = gate.state[idx + z];
    r.row = gate.rows[(int64_t)idx * DTH + min(lane, DTH - 1) + z];
    return r;
}

// Mask-gated detection: the same results as k_detect on every active centre
// (see k_gate_rows).  Tiles without an active centre are neither loaded nor
// computed; dense tiles run k_detect's body; on the other tiles the active
// centres, and the pixels whose coefficients they read (one pixel around
// each), are compacted into LDS work lists so that every lane of every wave
// does useful work in both phases.
__global__ __launch_bounds__(256, 3) void k_detect_gated(const float* __restrict__ pyr, const DetTile* __restrict__ tiles,
                                                      int ntiles, DetParams dp, GateParams gate,
                                                      cdvs_keypoint* __restrict__ cand,
                                                      int32_t* __restrict__ cand_cnt, int32_t* __restrict__ flags) {
    __shared__ __align__(16) float G[kScales][GH][GW];
    __shared__ float4 A[AH][AW];
    __shared__ uint16_t alist[AH * AW];
    __shared__ uint16_t clist[DTH * DTW];
    __shared__ int nlist;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int x = blockIdx.x % kXcds, slot = blockIdx.x / kXcds, nslot = gridDim.x / kXcds;
    const int per = ntiles / kXcds, rem = ntiles % kXcds;
    const int tbase = x * per + min(x, rem), cnt = per + (x < rem ? 1 : 0);
    if (slot >= cnt) return;   // uniform over the workgroup
    float4 vals[DNPER4];
    DetTile cur = as_uniform(fetch_tile(tiles, tbase + slot));
    RawGate gcur = fetch_gate(gate, tbase + slot);
    int scur = __builtin_amdgcn_readfirstlane(gcur.state);
    if (scur != kTileSkip) load_tile(pyr, cur, vals);
    RawTile rn = fetch_tile(tiles, tbase + min(slot + nslot, cnt - 1));
    RawGate gn = fetch_gate(gate, tbase + min(slot + nslot, cnt - 1));
    for (int tj = slot; tj < cnt; tj += nslot) {
        const int inn = tbase + min(tj + 2 * nslot, cnt - 1);
        const RawTile rnn = fetch_tile(tiles, inn);
        const RawGate gnn = fetch_gate(gate, inn);
        const bool has_next = tj + nslot < cnt;
        const DetTile nxt = as_uniform(rn);
        const int snxt = has_next ? __builtin_amdgcn_readfirstlane(gn.state) : kTileSkip;
        if (scur == kTileSkip) {
            if (snxt != kTileSkip) load_tile(pyr, nxt, vals);
        } else {
            __syncthreads();  // the previous tile is done with G, A and the lists
            store_tile(&G[0][0][0], vals);
            if (threadIdx.x == 0) nlist = 0;
            __syncthreads();
            if (snxt != kTileSkip) load_tile(pyr, nxt, vals);
            if (scur == kTileDense) {
                for (int t = threadIdx.x; t < AH * AW; t += blockDim.x) {
                    const int ay = t / AW, ax = t % AW;
                    A[ay][ax] = alpha_at(G, ay + 1, ax + 1 + GX, dp);
                }
                __syncthreads();
                float4* list = reinterpret_cast<float4*>(&G[0][0][0]);
                for (int it = 0; it < DTW * DTH / 256; ++it) {
                    const int q = threadIdx.x + it * 256;
                    const int cy = q / DTW, cx = q % DTW;
                    const int gx = cur.tx0 + cx, gy = cur.ty0 + cy;
                    float cs = 0.f, cp = 0.f, cpss = 0.f;
                    const bool pass = gx >= dp.border && gx <= cur.w - 1 - dp.border && gy >= dp.border &&
                                      gy <= cur.h - 1 - dp.border && centre_extremum(A, cy, cx, dp, cs, cp, cpss);
                    push_centre(pass, cs, cp, cpss, q, list, &nlist);
                }
                __syncthreads();
                refine_list(A, list, nlist, cur, dp, cand, cand_cnt, flags);
            } else {
                // lanes 0..15 of every wave hold the row masks
                const uint64_t myrow = lane < DTH ? gcur.row : 0ull;
                // centre list: row bases from a wave scan of the row counts
                const int rc = __popcll(myrow);
                const int rb = wave_excl_scan(rc);
                const int nc = __shfl(rb, DTH - 1) + __shfl(rc, DTH - 1);
                for (int cy = wave; cy < DTH; cy += 4) {
                    const uint64_t m = __shfl(myrow, cy);
                    const int base = __shfl(rb, cy);
                    if ((m >> lane) & 1)
                        clist[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)(cy * DTW + lane);
                }
                // coefficient list: alpha row ay is read by centre rows
                // ay-2..ay, alpha column ax by centre columns ax-2..ax
                const uint64_t r0 = __shfl(myrow, max(lane - 2, 0)), r1 = __shfl(myrow, max(lane - 1, 0));
                const uint64_t r2 = __shfl(myrow, min(lane, 63));
                uint64_t v = 0;
                if (lane < AH) {
                    if (lane - 2 >= 0 && lane - 2 < DTH) v |= r0;
                    if (lane - 1 >= 0 && lane - 1 < DTH) v |= r1;
                    if (lane < DTH) v |= r2;
                }
                const uint64_t vlo = v | (v << 1) | (v << 2);
                const uint32_t vhi = (uint32_t)(((v >> 62) | (v >> 63)) & 1u) | (uint32_t)(((v >> 63) & 1u) << 1);
                const int ac = __popcll(vlo) + __popc(vhi);
                const int ab = wave_excl_scan(ac);
                const int na = __shfl(ab, AH - 1) + __shfl(ac, AH - 1);
                for (int ay = wave; ay < AH; ay += 4) {
                    const uint64_t m = __shfl(vlo, ay);
                    const uint32_t mh = __shfl(vhi, ay);
                    const int base = __shfl(ab, ay);
                    if ((m >> lane) & 1)
                        alist[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)(ay * AW + lane);
                    if (lane < 2 && ((mh >> lane) & 1))
                        alist[base + __popcll(m) + (lane == 1 ? (int)(mh & 1u) : 0)] = (uint16_t)(ay * AW + DTW + lane);
                }
                __syncthreads();
                for (int i = threadIdx.x; i < na; i += blockDim.x) {
                    const int idx = alist[i];
                    const int ay = idx / AW, ax = idx % AW;
                    A[ay][ax] = alpha_at(G, ay + 1, ax + 1 + GX, dp);
                }
                __syncthreads();
                float4* list = reinterpret_cast<float4*>(&G[0][0][0]);
                for (int i0 = 0; i0 < nc; i0 += blockDim.x) {
                    const int i = i0 + threadIdx.x;
                    float cs = 0.f, cp = 0.f, cpss = 0.f;
                    int q = 0;
                    bool pass = false;
                    if (i < nc) {
                        q = clist[i];
                        pass = centre_extremum(A, q / DTW, q % DTW, dp, cs, cp, cpss);
                    }
                    push_centre(pass, cs, cp, cpss, q, list, &nlist);
                }
                __syncthreads();
                refine_list(A, list, nlist, cur, dp, cand, cand_cnt, flags);
            }
        }
        cur = nxt;
        gcur = gn;
        scur = snxt;
        rn = rnn;
        gn = gnn;
    }
}

__global__ void k_clear(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

constexpr int FIN_THREADS = 1024;
constexpr int FIN_PER = kCandCap / FIN_THREADS;  // candidates per thread

// Top-kCandCap selection by |p| for images with more candidates than the
// finalisation holds (one workgroup per image; the others return at once).
// The kCandCap-th largest |p| is found by a three-round radix select on the
// float bits of |p| (11, 11 and 10 bits; non-negative floats order like
// their bits), then every candidate above it and enough of those equal to it
// are copied out (in no particular order: the finalisation sorts).
__global__ __launch_bounds__(FIN_THREADS) void k_select(const cdvs_keypoint* __restrict__ cand,
                                                        const int32_t* __restrict__ cand_cnt,
                                                        const int64_t* __restrict__ cand_off,
                                                        const int32_t* __restrict__ cand_capv,
                                                        cdvs_keypoint* __restrict__ sel) {
    __shared__ int hist[2048];
    __shared__ uint32_t prefix_s, need_s;
    __shared__ int n_out, n_tie;
    const int img = blockIdx.x;
    const int n = min(cand_cnt[img], cand_capv[img]);
    if (n <= kCandCap) return;   // uniform over the workgroup
    const cdvs_keypoint* c = cand + cand_off[img];
    cdvs_keypoint* out = sel + (int64_t)img * kCandCap;
    if (threadIdx.x == 0) {
        prefix_s = 0u;
        need_s = kCandCap;
        n_out = 0;
        n_tie = 0;
    }
    uint32_t mask = 0u;   // bits of the threshold fixed so far
    const int shifts[3] = {21, 10, 0}, widths[3] = {11, 11, 10};
    for (int round = 0; round < 3; ++round) {
        const int sh = shifts[round], nb = 1 << widths[round];
        for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
        __syncthreads();
        const uint32_t prefix = prefix_s;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t key = __float_as_uint(fabsf(c[i].p));
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> sh) & (nb - 1)], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // walk the bins from the top until `need` keys are covered
            uint32_t need = need_s;
            int b = nb - 1;
            for (; b > 0 && (uint32_t)hist[b] < need; --b) need -= (uint32_t)hist[b];
            prefix_s = prefix | ((uint32_t)b << sh);
            need_s = need;   // keys still needed from bin b (the threshold's bin)
        }
        mask |= (uint32_t)(nb - 1) << sh;
        __syncthreads();
    }
    const uint32_t thr = prefix_s, ties = need_s;   // keep every key > thr and `ties` keys == thr
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t key = __float_as_uint(fabsf(c[i].p));
        bool take = key > thr;
        if (key == thr) take = atomicAdd(&n_tie, 1) < (int)ties;
        if (take) out[atomicAdd(&n_out, 1)] = c[i];
    }
}

// Ascending bitonic sort of npow (a power of two) 64-bit keys with 16-bit
// payloads in LDS by the whole workgroup.
__device__ __forceinline__ void bitonic_sort(unsigned long long* key, unsigned short* idx, int npow) {
    for (int size = 2; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < npow / 2; t += blockDim.x) {
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
}

// Stage C + canonical sort + top-k for one image per workgroup.  The
// candidates are first sorted by (octave, y) so that each one meets only the
// adjacent-octave candidates in a band of y around it (binary search, then a
// short scan) instead of every candidate of those octaves; the decisions are
// the same, as only pairs farther apart in y than the distance limit are
// skipped.  Then the survivors are sorted by the canonical key.
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const cdvs_keypoint* __restrict__ cand,
                                                          const int32_t* __restrict__ cand_cnt,
                                                          const int64_t* __restrict__ cand_off,
                                                          const int32_t* __restrict__ cand_capv,
                                                          const cdvs_keypoint* __restrict__ sel,
                                                          float ratio_lim, int topk, int kp_cap,
                                                          cdvs_keypoint* __restrict__ kp,
                                                          int32_t* __restrict__ count,
                                                          int32_t* __restrict__ flags) {
    // 128 KB: sort keys + payloads, then the records (x, y, sigma, p) in
    // (octave, y) order, then the final keys + payloads
    __shared__ float4 rec[kCandCap];
    __shared__ unsigned short perm[kCandCap];   // original index of each (octave, y)-sorted position
    __shared__ int seg[kMaxOctaves + 2];        // first sorted position of each octave
    __shared__ int n_alive;
    __shared__ uint32_t min_bits;               // smallest |p| (as bits) of a reduced image's set
    unsigned long long* key = reinterpret_cast<unsigned long long*>(rec);
    unsigned short* idx = reinterpret_cast<unsigned short*>(key + kCandCap);

    const int img = blockIdx.x;
    // an image with more candidates than the LDS holds was reduced to its
    // kCandCap strongest by k_select (exactly the ones stage C and the top-k
    // can keep: a candidate only ever loses to a stronger one)
    const int n_all = min(cand_cnt[img], cand_capv[img]);
    const cdvs_keypoint* c = n_all > kCandCap ? sel + (int64_t)img * kCandCap : cand + cand_off[img];
    const int n = min(n_all, kCandCap);
    const int tid = threadIdx.x;
    int npow = 1;
    while (npow < n) npow <<= 1;

    if (tid < kMaxOctaves + 2) seg[tid] = n;
    if (tid == 0) {
        n_alive = 0;
        min_bits = 0xffffffffu;
    }
    __syncthreads();
    uint32_t my_min = 0xffffffffu;
    for (int i = tid; i < npow; i += FIN_THREADS) {
        // y >= 0, so its float bits order like the value
        key[i] = i < n ? ((unsigned long long)c[i].octave << 32) | __float_as_uint(c[i].y) : ~0ull;
        idx[i] = (unsigned short)i;
        if (i < n) my_min = min(my_min, __float_as_uint(fabsf(c[i].p)));
    }
    if (n_all > kCandCap) atomicMin(&min_bits, my_min);
    __syncthreads();
    bitonic_sort(key, idx, npow);
    for (int i = tid; i < n; i += FIN_THREADS) {
        perm[i] = idx[i];
        const int o = (int)(key[i] >> 32);
        const int prev = i == 0 ? -1 : (int)(key[i - 1] >> 32);
        for (int oo = prev + 1; oo <= o; ++oo) seg[oo] = i;
    }
    __syncthreads();   // keys are read; the records overwrite them
    for (int i = tid; i < n; i += FIN_THREADS) {
        const cdvs_keypoint a = c[perm[i]];
        rec[i] = make_float4(a.x, a.y, a.sigma, a.p);
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
            int ao = 0;
            while (ao + 1 < kMaxOctaves + 1 && seg[ao + 1] <= i) ++ao;
            const float aa = fabsf(a.w);
            bool alive = true;
            for (int d = -1; d <= 1 && alive; d += 2) {
                const int o2 = ao + d;
                if (o2 < 0 || o2 >= kMaxOctaves) continue;
                const float lim = (float)(1 << max(ao, o2));
                const float lim2 = lim * lim;
                // the band searched is one pixel wider than the limit, so
                // rounding here cannot drop a pair the exact test keeps
                const float ylo = a.y - (lim + 1.f), yhi = a.y + (lim + 1.f);
                int lo = seg[o2], hi = seg[o2 + 1];
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (rec[mid].y < ylo) lo = mid + 1;
                    else hi = mid;
                }
                for (int jj = lo; jj < seg[o2 + 1]; ++jj) {
                    const float4 b = rec[jj];
                    if (b.y > yhi) break;
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
                const cdvs_keypoint& r = c[perm[i]];
                kk[j] = ((unsigned long long)(~__float_as_uint(aa)) << 32) |
                        ((unsigned long long)ao << 28) | ((unsigned long long)r.iy << 14) |
                        (unsigned long long)r.ix;
            }
        }
    }
    if (local_alive) atomicAdd(&n_alive, local_alive);
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
    bitonic_sort(key, idx, npow);

    const int limit = min(topk > 0 ? topk : kp_cap, kp_cap);
    const int m = min(n_alive, limit);
    for (int r = tid; r < m; r += blockDim.x) kp[(int64_t)img * kp_cap + r] = c[perm[idx[r]]];
    if (tid == 0) {
        count[img] = m;
        // A reduced image's output is exact when its last kept keypoint is
        // stronger than every candidate k_select dropped: each kept one was
        // judged against all candidates at least as strong, and no dropped
        // candidate could rank among them.  Otherwise the image is flagged.
        if (n_all > kCandCap && limit > 0) {
            const bool exact = n_alive >= limit && ~(uint32_t)(key[limit - 1] >> 32) > min_bits;
            if (!exact) atomicOr(flags, kFlagSelectInexact);
        }
    }
}

}  // namespace

hipError_t launch_clear(int32_t* p, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_detect(const float* pyr, const DetTile* tiles, int ntiles, int grid, const DetParams& dp,
                         const GateParams& gate, cdvs_keypoint* cand, int32_t* cand_cnt, int32_t* flags,
                         hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    // a multiple of the XCD count, no larger than needed
    int g = std::min(grid, (ntiles + kXcds - 1) / kXcds * kXcds);
    g = std::max(kXcds, g / kXcds * kXcds);
    if (gate.mask)
        hipLaunchKernelGGL(k_detect_gated, dim3(g), dim3(256), 0, stream, pyr, tiles, ntiles, dp, gate, cand, cand_cnt,
                           flags);
    else
        hipLaunchKernelGGL(k_detect, dim3(g), dim3(256), 0, stream, pyr, tiles, ntiles, dp, cand, cand_cnt, flags);
    return hipGetLastError();
}

hipError_t launch_gate_rows(const DetTile* tiles, int ntiles, const DetParams& dp, const GateParams& gate,
                            uint64_t* rows, int32_t* state, hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gate_rows, dim3((ntiles + 3) / 4), dim3(256), 0, stream, tiles, ntiles, dp, gate, rows, state);
    return hipGetLastError();
}

hipError_t launch_detect_strips(const float* pyr, const DetTile* strips, int nstrips, const DetParams& dp,
                               cdvs_keypoint* cand, int32_t* cand_cnt, int32_t* flags, hipStream_t stream) {
    if (nstrips <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_detect_strip, dim3((nstrips + 3) / 4), dim3(256), 0, stream, pyr, strips, nstrips, dp, cand,
                       cand_cnt, flags);
    return hipGetLastError();
}

hipError_t launch_select(const cdvs_keypoint* cand, const int32_t* cand_cnt, const int64_t* cand_off,
                         const int32_t* cand_capv, int n_images, cdvs_keypoint* sel, hipStream_t stream) {
    if (n_images <= 0 || !sel) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3(n_images), dim3(FIN_THREADS), 0, stream, cand, cand_cnt, cand_off, cand_capv, sel);
    return hipGetLastError();
}

hipError_t launch_finalize(const cdvs_keypoint* cand, const int32_t* cand_cnt, const int64_t* cand_off,
                           const int32_t* cand_capv, const cdvs_keypoint* sel, int n_images, float dedup_ratio,
                           int topk, int kp_cap, cdvs_keypoint* kp, int32_t* count, int32_t* flags,
                           hipStream_t stream) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(n_images), dim3(FIN_THREADS), 0, stream, cand, cand_cnt, cand_off, cand_capv,
                       sel, dedup_ratio, topk, kp_cap, kp, count, flags);
    return hipGetLastError();
}

}  // namespace cdvs
