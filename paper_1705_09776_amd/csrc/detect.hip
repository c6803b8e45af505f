// ALP keypoint detection on gfx950 (Sec. III-A, Eqs. (2)-(3); Sec. IV-A,
// Algorithm 1 stages A-C).
//
// k_detect_strip: one wave per strip of 60 x 48 centres of one (image,
//   octave), all octaves of all images in one launch; the wave streams the
//   five Gaussian images down its strip in registers (details at the kernel).
//   Per centre: scale-normalised 5-point Laplacians, the four ALP
//   coefficients, extremal scale, contrast test, strict 8-neighbour test at
//   that scale, one quadratic refinement step; survivors go to the image's
//   candidate list with one ballot and one atomic per pass.  With a cell
//   mask (the learned gate) only the centres of active cells are examined
//   and strips without any are skipped before loading anything.
// k_select (images with more candidates than k_finalize holds): their
//   strongest kCandCap by |p|.
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
// |p| has a maximum (p p'' < 0); larger |p| wins, then the smaller s.  The
// roots of p'(s) = A s^2 + B s + C come from the stable quadratic formula,
// s0 = q / A and s1 = C / q; when A = 0, q = -B and s1 is the linear root.
// Both candidates are evaluated and the choice is made by selects (no
// branches: every lane of a wave runs this), with correctly rounded
// quotients (the extremal scale is ill-conditioned, so the quotients are
// not replaced by reciprocal approximations).
__device__ __forceinline__ bool alp_extremum(const float4 a, float lo, float hi, float& s_out, float& p_out,
                                             float& pss_out) {
    const float A = 3.f * a.w, B = 2.f * a.z, C = a.y;
    const bool lin = A == 0.f;
    const float disc = B * B - 4.f * A * C;
    const float sq = __builtin_amdgcn_sqrtf(fmaxf(disc, 0.f));   // hardware square root (1 ulp)
    const float q = (B >= 0.f) ? -(B + sq) * 0.5f : -(B - sq) * 0.5f;
    const float s0 = q / A;
    const float s1 = C / (lin ? -B : q);
    const bool real = lin || disc >= 0.f;
    const float p0 = horner(a, s0), p1 = horner(a, s1);
    const float pss0 = 6.f * a.w * s0 + 2.f * a.z, pss1 = 6.f * a.w * s1 + 2.f * a.z;
    const bool ok0 = real & !lin & (s0 >= lo) & (s0 < hi) & (p0 * pss0 < 0.f);
    const bool ok1 = real & (s1 >= lo) & (s1 < hi) & (p1 * pss1 < 0.f);
    const float a0 = fabsf(p0), a1 = fabsf(p1);
    const bool take1 = ok1 & (!ok0 | (a1 > a0) | ((a1 == a0) & (s1 < s0)));
    // without an extremum the outputs are left as they fall (possibly not
    // finite): they then only feed this centre's own tests, which it fails
    s_out = take1 ? s1 : s0;
    p_out = take1 ? p1 : p0;
    pss_out = take1 ? pss1 : pss0;
    return ok0 | ok1;
}

// 5-point Laplacian sum (up + down + left + right - 4 centre), in one fixed
// order of operations for the plain and the gated detection.
__device__ __forceinline__ float lap5(float c, float up, float dn, float lf, float rt) {
    float s = up + dn;
    s = s + lf;
    s = s + rt;
    s = s - 4.f * c;
    return s;
}

// Adds scale k's normalised Laplacian sigma_k^2 lap to the ALP coefficients
// (sigma_k^2 is folded into the fitting weights on the host).
__device__ __forceinline__ void alpha_acc(float4& a, float lap, int k, const DetParams& dp) {
    a.x = fmaf(dp.bsig[k][0], lap, a.x);
    a.y = fmaf(dp.bsig[k][1], lap, a.y);
    a.z = fmaf(dp.bsig[k][2], lap, a.z);
    a.w = fmaf(dp.bsig[k][3], lap, a.w);
}

struct Cand {
    float s, p, pss, ox, oy, pr, rho;
};

// Strict extremum of the centre value p = v[4] against the eight
// neighbours' cubics v[] evaluated at the centre's scale (Algorithm 1 stage A).
// (All eight below p for a maximum, above it for a minimum: compared through
// their max and min, without branches; mn > p is tested as -mn < -p = |p|,
// so one float select and one comparison decide both cases exactly; the
// values are finite.)
__device__ __forceinline__ bool strict_extremum(const float (&v)[9], float p) {
    float mx = v[0], mn = v[0];
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (i != 4) {
            mx = fmaxf(mx, v[i]);
            mn = fminf(mn, v[i]);
        }
    return (p > 0.f ? mx : -mn) < fabsf(p);
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

// ---------------------------------------------------------------------------
// k_detect_strip: the detection, one wave per strip of kStripW
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
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v) {  // lane l gets lane l+1's value (lane 63: 0)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

struct StripRow {
    float g[kScales];
};

// The five planes of a strip's (image, octave): their bases are the same in
// every lane and kept in scalar registers, and a lane reads a row as one
// 32-bit byte offset from each (an octave's planes span less than 2^32
// bytes, as sides are at most CDVS_MAX_SIDE), so a row costs one vector add
// for its address instead of a 64-bit address per plane.
struct StripPlanes {
    const char* base[kScales];
    uint32_t col4;   // this lane's (clamped) column, in bytes
};

__device__ __forceinline__ StripPlanes strip_planes(const float* __restrict__ pyr, const DetTile& job, int gx) {
    StripPlanes sp;
    // (the offset, not the pointer, goes through the scalar unit: a pointer
    // rebuilt from an integer would lose its global address space)
#pragma unroll
    for (int k = 0; k < kScales; ++k) {
        const uint64_t o = (uint64_t)(job.plane0 + (int64_t)k * job.plane_stride);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)o);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(o >> 32));
        sp.base[k] = reinterpret_cast<const char*>(pyr + (int64_t)(((uint64_t)hi << 32) | lo));
    }
    sp.col4 = (uint32_t)clampi(gx, 0, job.w - 1) * 4u;
    return sp;
}

// Plane row y (clamped to the image) of this lane's column.
__device__ __forceinline__ void load_row(const StripPlanes& sp, const DetTile& job, int y, StripRow& r) {
    const uint32_t off = (uint32_t)clampi(y, 0, job.h - 1) * (uint32_t)job.pitch * 4u + sp.col4;
#pragma unroll
    for (int k = 0; k < kScales; ++k) r.g[k] = *reinterpret_cast<const float*>(sp.base[k] + off);
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
    const bool found = alp_extremum(aM, dp.lo, dp.hi, s, p, pss);
    const bool pass = col_ok & found & (fabsf(p) >= dp.contrast);   // no branch: every lane evaluates
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
    const bool keep = pass & strict_extremum(v, p);   // both evaluated: no branch
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

// GATED: an octave-o centre (x, y) is examined only when bit o of the mask
// cell holding (x 2^o, y 2^o) / 4 is set, unless more than gate.fmax of the
// image's cells have bit o set, or o is beyond the gate's kCnnHeads bits
// (then the octave is examined densely).
template <bool GATED>
__device__ __forceinline__ void detect_strip(const float* __restrict__ pyr, const DetTile& job, const DetParams& dp,
                                             const GateParams& gate, float (*q)[kQCap],
                                             cdvs_keypoint* __restrict__ cand, int32_t* __restrict__ cand_cnt,
                                             int32_t* __restrict__ flags) {
    static_assert(kStripH <= 64, "one activity bit per strip row");
    const int lane = threadIdx.x & 63;
    const int x0 = job.tx0, y0 = job.ty0;
    const int xend = min(x0 + kStripW, job.w - dp.border), yend = min(y0 + kStripH, job.h - dp.border);
    const int gx = x0 - 2 + lane;
    const bool col_ok = lane >= 2 && gx < xend;
    // bit i: this lane's centre on row y0 + i is examined
    uint64_t rows_on = ~0ull;
    if constexpr (GATED) {
        const CnnImage cg = gate.cells[job.image];
        const bool dense =
            job.octave >= kCnnHeads ||
            (float)gate.active[job.image * kMaxOctaves + job.octave] > gate.fmax * (float)(cg.H4 * cg.W4);
        if (!dense) {
            rows_on = 0ull;
            if (col_ok) {
                const uint8_t* m = gate.mask + cg.cell0 + min((gx << job.octave) >> 2, cg.W4 - 1);
                for (int y = y0; y < yend; ++y) {
                    const int cy = min((y << job.octave) >> 2, cg.H4 - 1);
                    rows_on |= (uint64_t)((m[(int64_t)cy * cg.W4] >> job.octave) & 1) << (y - y0);
                }
            }
            if (!__ballot(rows_on != 0ull)) return;   // nothing active: the strip is not even loaded
        }
    }
    const StripPlanes col = strip_planes(pyr, job, gx);
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
                strip_centres(a[r % 3], a[(r + 1) % 3], a[(r + 2) % 3], col_ok && ((rows_on >> (y + r - y0)) & 1ull),
                              gx, y + r, q, qn, job, dp, cand, cand_cnt, flags);
        }
    }
    strip_drain(q, qn, job, dp, cand, cand_cnt, flags);
}

// Requests one strip index from this XCD's work counter; the value arrives
// in lane 0 and is read (made uniform) only when it is needed.  (An
// increment rather than an add: the compiler rewrites a single-lane add into
// a wave-wide one whose result it consumes at once, stalling on the round
// trip; the counter never comes near the wrap limit.)
__device__ __forceinline__ int fetch_strip(int32_t* __restrict__ ctr) {
    unsigned t = 0u;
    if ((threadIdx.x & 63) == 0) t = atomicInc(reinterpret_cast<unsigned*>(ctr), 0xffffffffu);
    return (int)t;
}

// Two launch forms (picked by the autotuner):
// PERSISTENT = false: one wave per strip, the hardware dispatching the
//   workgroups (xcd_remap gives each XCD one contiguous range of strips).
// PERSISTENT = true: the grid (a multiple of 8, sized to the waves the chip
//   holds) is split evenly over the XCDs, and every XCD owns one contiguous
//   range of strips with a work counter in `work` (zeroed before the
//   launch); each wave pulls its next strip from the counter until the range
//   is used up, so uneven strips (octaves, ragged images, skipped gated
//   strips) balance by themselves.  The next index is requested when a
//   strip starts and read when it ends, so the atomic's round trip overlaps
//   the strip's work.
// Either way neighbouring strips run close together in time on one XCD and
// share their halo rows through its L2.
template <bool GATED, bool PERSISTENT>
__global__ __launch_bounds__(256) void k_detect_strip(const float* __restrict__ pyr, const DetTile* __restrict__ strips,
                                                      int nstrips, DetParams dp, GateParams gate,
                                                      int32_t* __restrict__ work, cdvs_keypoint* __restrict__ cand,
                                                      int32_t* __restrict__ cand_cnt, int32_t* __restrict__ flags) {
    __shared__ float queue[4][kQFields][kQCap];
    const int wave = threadIdx.x >> 6;
    if constexpr (!PERSISTENT) {
        const int sidx = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * 4 + wave);
        if (sidx >= nstrips) return;   // uniform over the wave; there are no barriers
        const DetTile job = strips[sidx];
        detect_strip<GATED>(pyr, job, dp, gate, queue[wave], cand, cand_cnt, flags);
    } else {
        const int x = blockIdx.x % kXcds;
        const int per = nstrips / kXcds, rem = nstrips % kXcds;
        const int base = x * per + min(x, rem), cnt = per + (x < rem ? 1 : 0);
        int32_t* ctr = work + x;
        int pending = fetch_strip(ctr);
        for (;;) {
            const int t = __builtin_amdgcn_readfirstlane(pending);
            if (t >= cnt) break;   // uniform over the wave; there are no barriers
            pending = fetch_strip(ctr);
            const DetTile job = strips[base + t];
            detect_strip<GATED>(pyr, job, dp, gate, queue[wave], cand, cand_cnt, flags);
        }
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

// One compare-exchange of a bitonic stage of block size `size` at distance
// S < 64 for the (key, payload) of element i held by this lane, whose
// partner (i ^ S) is in lane ^ S: the lower index keeps the smaller key in
// an ascending block, the larger in a descending one (equal keys stay where
// they are).  Both comparisons are made and one is selected, so no lane
// branches.
template <int S>
__device__ __forceinline__ void bitonic_lane_step(unsigned long long& k, int& p, int i, int size) {
    const unsigned long long o = lane_xor64<S>(k);
    const int op = (int)lane_xor<S>((uint32_t)p);
    const bool want_min = ((i & size) == 0) == ((i & S) == 0);
    const bool lt = o < k, gt = k < o;
    const bool take = (want_min & lt) | (!want_min & gt);
    k = take ? o : k;
    p = take ? op : p;
}

// The distances 32, 16, .., 1 (those below `size`) of one bitonic stage
// for both of the lane's elements.
__device__ __forceinline__ void bitonic_lane_steps(unsigned long long& k0, int& p0, int i0, unsigned long long& k1,
                                                   int& p1, int i1, int size) {
#define CDVS_STEP(S)                                   \
    if (size > S) {                                    \
        bitonic_lane_step<S>(k0, p0, i0, size);        \
        bitonic_lane_step<S>(k1, p1, i1, size);        \
    }
    CDVS_STEP(32) CDVS_STEP(16) CDVS_STEP(8) CDVS_STEP(4) CDVS_STEP(2) CDVS_STEP(1)
#undef CDVS_STEP
}

// The steps at distances below 128 of bitonic block sizes first..last on
// the 128-entry chunks of [0, npow): each wave takes whole chunks, two
// entries per lane (c*128 + lane and c*128 + 64 + lane) in registers.
__device__ __forceinline__ void bitonic_chunk_steps(unsigned long long* key, unsigned short* idx, int npow, int first,
                                                    int last) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = wave; c < npow / 128; c += nw) {
        const int i0 = 128 * c + lane, i1 = i0 + 64;
        unsigned long long k0 = key[i0], k1 = key[i1];
        int p0 = idx[i0], p1 = idx[i1];
        for (int size = first; size <= last; size <<= 1) {
            if (size >= 128) {   // distance 64: the lane's own pair, one direction for both
                const bool asc = (i0 & size) == 0;
                if (asc ? (k0 > k1) : (k0 < k1)) {
                    const unsigned long long tk = k0;
                    k0 = k1;
                    k1 = tk;
                    const int tp = p0;
                    p0 = p1;
                    p1 = tp;
                }
            }
            bitonic_lane_steps(k0, p0, i0, k1, p1, i1, size);
        }
        key[i0] = k0;
        key[i1] = k1;
        idx[i0] = (unsigned short)p0;
        idx[i1] = (unsigned short)p1;
    }
}

// Ascending bitonic sort of npow (a power of two, at least 128) 64-bit keys
// with 16-bit payloads in LDS by the whole workgroup: block sizes up to 128
// entirely in registers (lane shuffles), then for each larger size its
// distances of 128 and more through LDS with a barrier each, the rest in
// registers.
__device__ void bitonic_sort(unsigned long long* key, unsigned short* idx, int npow) {
    bitonic_chunk_steps(key, idx, npow, 2, 128);
    __syncthreads();
    for (int size = 256; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride >= 128; stride >>= 1) {
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
        bitonic_chunk_steps(key, idx, npow, size, size);
        __syncthreads();
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
    int npow = 128;   // the sort works on whole 128-entry chunks (padding sorts last)
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

hipError_t launch_detect_strips(const float* pyr, const DetTile* strips, int nstrips, int variant, int grid,
                                const DetParams& dp, const GateParams& gate, int32_t* work, cdvs_keypoint* cand,
                                int32_t* cand_cnt, int32_t* flags, hipStream_t stream) {
    if (nstrips <= 0) return hipSuccess;
#define DETECT_LAUNCH(G, P, NB)                                                                                    \
    hipLaunchKernelGGL((k_detect_strip<G, P>), dim3(NB), dim3(256), 0, stream, pyr, strips, nstrips, dp, gate, work, \
                       cand, cand_cnt, flags)
    if (variant == kDetectPersistent) {
        // a multiple of the XCD count, no larger than one wave per strip
        int g = std::min(grid, (nstrips + 4 * kXcds - 1) / (4 * kXcds) * kXcds);
        g = std::max(kXcds, g / kXcds * kXcds);
        if (gate.mask)
            DETECT_LAUNCH(true, true, g);
        else
            DETECT_LAUNCH(false, true, g);
    } else {
        const int nb = (nstrips + 3) / 4;
        if (gate.mask)
            DETECT_LAUNCH(true, false, nb);
        else
            DETECT_LAUNCH(false, false, nb);
    }
#undef DETECT_LAUNCH
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
