// Host side of the gfx950 CDVS library: argument validation, the batch
// layout (pyramid plane offsets, per-octave tile lists), the constant blocks
// handed to the kernels, and the C ABI of include/cdvs.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <fstream>
#include <functional>
#include <mutex>
#include <thread>
#include <sstream>
#include <string>
#include <vector>

#include "cdvs_internal.h"

using namespace cdvs;

struct cdvs_ctx {
    cdvs_params params{};
    int n = 0;
    int kp_cap = 0;
    std::vector<cdvs_image_desc> images;
    std::vector<int> octaves;                  // per image
    std::vector<OctGeom> geom;                 // [n][kMaxOctaves]
    std::vector<OctJob> jobs;                  // grouped by octave
    int max_oct = 0;
    int job_start[kMaxOctaves + 1] = {};
    int blur_tiles[kBlurTilings][kMaxOctaves] = {};
    int blur_variant = 1;    // scale-plane tile variant (cdvs_autotune; 128 x 16 measured best untuned)
    int detect_variant = 0;  // detection launch form (cdvs_autotune)
    int64_t pyr_floats = 0;
    Taps taps{};
    DetParams det{};
    OriParams ori{};
    DescParams desc{};
    float dedup_ratio = 0.f;
    int wgrad_grid = 0;   // grid of the CNN weight-gradient kernels
    int detect_grid = 0;  // persistent detection grid (workgroups)
    // surrogate CNN cell grid
    std::vector<CnnImage> cnn;
    int64_t ncells = 0;
    int cnn_tiles = 0, cnn_chunks = 0, cnn_ftiles = 0;
    CnnImage* d_cnn = nullptr;
    int32_t* d_active = nullptr;  // [n][kMaxOctaves] active mask cells
    short* d_cnn_frag = nullptr;  // packed weight fragments of the fused inference kernel
    float* d_scfv_prep = nullptr; // SCFV per-call model constants (kScfvPrepFloats)
    int32_t* d_wh = nullptr;      // per image: width, height
    cdvs_image_desc* d_img = nullptr;  // the image table (front-end output layout)
    // BMLoG variant: per octave, (job, bx, by) of every block; transfer functions
    std::vector<int32_t> bm_blocks;
    int bm_start[kMaxOctaves] = {}, bm_count[kMaxOctaves] = {};
    int32_t* d_bm_blocks = nullptr;
    float* d_bm_H = nullptr;
    float bm_H[kBmTransfers * kBmN] = {};
    // device
    OctJob* d_jobs = nullptr;
    std::vector<int32_t> blur_owner;           // [variant][octave][tile] -> job (relative to job_start[octave])
    int blur_owner_start[kBlurTilings][kMaxOctaves] = {};
    int32_t* d_blur_owner = nullptr;
    std::vector<int32_t> cnn_owner;            // fused CNN tile -> image
    int32_t* d_cnn_owner = nullptr;
    std::vector<DetTile> strips;   // ungated detection: image-major, then octave, then row-major strips
    DetTile* d_strips = nullptr;
    OctGeom* d_geom = nullptr;
    cdvs_keypoint* d_cand = nullptr;           // per image: cand_cap[i] records from cand_off[i]
    std::vector<int64_t> cand_off;
    std::vector<int32_t> cand_cap;
    int64_t* d_cand_off = nullptr;
    int32_t* d_cand_capv = nullptr;
    cdvs_keypoint* d_sel = nullptr;            // [image][kCandCap] strongest candidates (only when needed)
    int32_t* d_cand_cnt = nullptr;             // n per-image counts, then kXcds detection work counters
    cdvs_keypoint* d_ori = nullptr;
    int32_t* d_ori_cnt = nullptr;
    int32_t* d_flags = nullptr;
    std::string err;
    // event brackets (cdvs_profile_*)
    bool prof = false;
    std::vector<hipEvent_t> ev;       // 2 per bracket
    std::vector<int> ev_id;           // kernel id per bracket
    int ev_used = 0;
    // captured pass (cdvs_graph_*)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
};

namespace {

thread_local std::string g_create_err;

cdvs_status fail(cdvs_ctx* ctx, cdvs_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_err = buf;
    return st;
}

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int count_octaves(int w, int h, int min_side) {
    int n = 1;
    while (std::min(w, h) >= min_side) {
        w = (w + 1) / 2;
        h = (h + 1) / 2;
        ++n;
    }
    return n;
}

// Gaussian taps exp(-p^2 / 2 s^2), |p| <= r, normalised to sum 1 (double),
// stored as float.
void make_taps(double s, int r, float* g) {
    double e[2 * kMaxR + 1], sum = 0.0;
    for (int p = -r; p <= r; ++p) {
        e[p + r] = exp(-(double)(p * p) / (2.0 * s * s));
        sum += e[p + r];
    }
    for (int i = 0; i < 2 * r + 1; ++i) g[i] = (float)(e[i] / sum);
}

// Least-squares cubic through (sigma_k, L_k), k = 0..4: coefficients
// beta[k][i] of alpha_i = sum_k beta[k][i] L_k, i.e. (V^T V)^-1 V^T with
// V_{k,i} = sigma_k^i, solved by Gauss-Jordan elimination in long double.
void make_beta(const double* sig, float beta[kScales][4]) {
    long double M[4][4 + kScales];
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) {
            long double a = 0;
            for (int k = 0; k < kScales; ++k) a += powl(sig[k], i) * powl(sig[k], j);
            M[i][j] = a;
        }
        for (int k = 0; k < kScales; ++k) M[i][4 + k] = powl(sig[k], i);
    }
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabsl(M[r][c]) > fabsl(M[piv][c])) piv = r;
        if (piv != c)
            for (int j = 0; j < 4 + kScales; ++j) {
                long double t = M[c][j];
                M[c][j] = M[piv][j];
                M[piv][j] = t;
            }
        long double d = M[c][c];
        for (int j = 0; j < 4 + kScales; ++j) M[c][j] /= d;
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            long double f = M[r][c];
            for (int j = 0; j < 4 + kScales; ++j) M[r][j] -= f * M[c][j];
        }
    }
    for (int k = 0; k < kScales; ++k)
        for (int i = 0; i < 4; ++i) beta[k][i] = (float)M[i][4 + k];
}

constexpr int kMaxBrackets = 16384;

// Brackets one kernel launch with events when profiling is on.
struct Bracket {
    cdvs_ctx* c;
    hipStream_t s;
    int slot = -1;
    Bracket(cdvs_ctx* ctx, int id, hipStream_t stream) : c(ctx), s(stream) {
        if (c->prof && c->ev_used < kMaxBrackets) {
            slot = c->ev_used++;
            c->ev_id[slot] = id;
            (void)hipEventRecord(c->ev[2 * slot], s);
        }
    }
    ~Bracket() {
        if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], s);
    }
};

#define HIP_OR_FAIL(ctx, expr)                                                                  \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(ctx, CDVS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" {

cdvs_params cdvs_default_params(void) {
    cdvs_params p;
    memset(&p, 0, sizeof(p));
    p.version = CDVS_PARAMS_VERSION;
    p.sigma0 = 1.6f;
    p.intervals = 4;
    p.min_side = 32;
    p.contrast = 1.5f;
    p.edge_r = 10.f;
    p.border = 4;
    p.max_offset = 0.5f;
    p.dedup_dlog2 = 0.25f;
    p.ori_radius = 3.96f;
    p.ori_wsigma = 1.5f;
    p.ori_peak = 0.8f;
    p.max_ori = 4;
    p.desc_cell = 3.f;
    p.desc_radius = 6.f;
    p.desc_wsigma = 6.f;
    p.desc_clamp = 0.2f;
    p.topk = 1000;
    p.mask_fmax = 0.6f;
    return p;
}

cdvs_status cdvs_validate(const cdvs_params* p, const cdvs_image_desc* im, int32_t n, int32_t kp_cap, char* msg,
                          int32_t msg_len) {
    char buf[256] = {0};
    cdvs_status st = CDVS_OK;
#define BAD(code, ...)                             \
    do {                                           \
        snprintf(buf, sizeof(buf), __VA_ARGS__);   \
        st = code;                                 \
        goto done;                                 \
    } while (0)
    if (!p) BAD(CDVS_ERR_ARG, "params is NULL");
    if (p->version != CDVS_PARAMS_VERSION) BAD(CDVS_ERR_VERSION, "params.version %d != %d", p->version, CDVS_PARAMS_VERSION);
    if (fabsf(p->sigma0 - 1.6f) > 1e-6f || p->intervals != 4)
        BAD(CDVS_ERR_ARG, "kernels are compiled for sigma0 = 1.6 and intervals = 4");
    if (p->min_side < 8) BAD(CDVS_ERR_ARG, "min_side %d < 8", p->min_side);
    if (!(p->contrast >= 0.f)) BAD(CDVS_ERR_ARG, "contrast must be >= 0");
    if (!(p->edge_r > 0.f)) BAD(CDVS_ERR_ARG, "edge_r must be > 0");
    if (p->border < 1) BAD(CDVS_ERR_ARG, "border must be >= 1");
    if (!(p->max_offset > 0.f)) BAD(CDVS_ERR_ARG, "max_offset must be > 0");
    if (!(p->dedup_dlog2 >= 0.f)) BAD(CDVS_ERR_ARG, "dedup_dlog2 must be >= 0");
    if (!(p->ori_radius > 0.f) || !(p->ori_radius <= 8.f)) BAD(CDVS_ERR_ARG, "ori_radius must be in (0, 8]");
    if (!(p->ori_wsigma > 0.f)) BAD(CDVS_ERR_ARG, "ori_wsigma must be > 0");
    if (!(p->ori_peak > 0.f) || !(p->ori_peak <= 1.f)) BAD(CDVS_ERR_ARG, "ori_peak must be in (0, 1]");
    if (p->max_ori < 1 || p->max_ori > kMaxOri) BAD(CDVS_ERR_ARG, "max_ori must be in 1..%d", kMaxOri);
    if (!(p->desc_cell > 0.f) || !(p->desc_radius > 0.f) || !(p->desc_radius <= 12.f) || !(p->desc_wsigma > 0.f))
        BAD(CDVS_ERR_ARG, "descriptor geometry must be positive (radius <= 12)");
    if (!(p->desc_clamp > 0.f)) BAD(CDVS_ERR_ARG, "desc_clamp must be > 0");
    if (kp_cap < 1 || kp_cap > CDVS_MAX_KP_CAPACITY)
        BAD(CDVS_ERR_SHAPE, "kp_capacity %d outside 1..%d", kp_cap, CDVS_MAX_KP_CAPACITY);
    if (p->topk > kp_cap) BAD(CDVS_ERR_ARG, "topk %d > kp_capacity %d", p->topk, kp_cap);
    if (!(p->mask_fmax >= 0.f) || !(p->mask_fmax <= 1.f)) BAD(CDVS_ERR_ARG, "mask_fmax must be in [0, 1]");
    if (n < 1 || n > CDVS_MAX_IMAGES) BAD(CDVS_ERR_SHAPE, "n_images %d outside 1..%d", n, CDVS_MAX_IMAGES);
    if (!im) BAD(CDVS_ERR_ARG, "images is NULL");
    for (int i = 0; i < n; ++i) {
        const cdvs_image_desc& d = im[i];
        if (d.width < CDVS_MIN_SIDE || d.height < CDVS_MIN_SIDE || d.width > CDVS_MAX_SIDE || d.height > CDVS_MAX_SIDE)
            BAD(CDVS_ERR_SHAPE, "image %d: %dx%d outside %d..%d per side", i, d.width, d.height, CDVS_MIN_SIDE,
                CDVS_MAX_SIDE);
        if (d.pitch < d.width) BAD(CDVS_ERR_SHAPE, "image %d: pitch %d < width %d", i, d.pitch, d.width);
        if (d.offset < 0) BAD(CDVS_ERR_SHAPE, "image %d: negative offset", i);
        if (count_octaves(d.width, d.height, p->min_side) > kMaxOctaves)
            BAD(CDVS_ERR_SHAPE, "image %d: more than %d octaves", i, kMaxOctaves);
    }
#undef BAD
done:
    if (msg && msg_len > 0) {
        strncpy(msg, buf, (size_t)msg_len - 1);
        msg[msg_len - 1] = 0;
    }
    return st;
}

const char* cdvs_last_error(const cdvs_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

void cdvs_ctx_destroy(cdvs_ctx* ctx) {
    if (!ctx) return;
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto& e : ctx->ev) (void)hipEventDestroy(e);
    (void)hipFree(ctx->d_jobs);
    (void)hipFree(ctx->d_strips);
    (void)hipFree(ctx->d_blur_owner);
    (void)hipFree(ctx->d_cnn_owner);
    (void)hipFree(ctx->d_geom);
    (void)hipFree(ctx->d_cand);
    (void)hipFree(ctx->d_cand_off);
    (void)hipFree(ctx->d_cand_capv);
    (void)hipFree(ctx->d_sel);
    (void)hipFree(ctx->d_cand_cnt);
    (void)hipFree(ctx->d_ori);
    (void)hipFree(ctx->d_ori_cnt);
    (void)hipFree(ctx->d_flags);
    (void)hipFree(ctx->d_cnn);
    (void)hipFree(ctx->d_active);
    (void)hipFree(ctx->d_cnn_frag);
    (void)hipFree(ctx->d_scfv_prep);
    (void)hipFree(ctx->d_wh);
    (void)hipFree(ctx->d_img);
    (void)hipFree(ctx->d_bm_blocks);
    (void)hipFree(ctx->d_bm_H);
    delete ctx;
}

static cdvs_status build_layout(cdvs_ctx* c) {
    const cdvs_params& p = c->params;
    c->octaves.resize(c->n);
    c->geom.assign((size_t)c->n * kMaxOctaves, OctGeom{0, 0, 0, 0, 0});
    std::vector<std::vector<OctJob>> per_oct(kMaxOctaves);
    int64_t off = 0;
    for (int i = 0; i < c->n; ++i) {
        const cdvs_image_desc& d = c->images[i];
        const int no = count_octaves(d.width, d.height, p.min_side);
        c->octaves[i] = no;
        c->max_oct = std::max(c->max_oct, no);
        int w = d.width, h = d.height;
        int64_t plane0[kMaxOctaves];
        int pitch[kMaxOctaves], stride[kMaxOctaves], ws[kMaxOctaves], hs[kMaxOctaves];
        for (int o = 0; o < no; ++o) {
            ws[o] = w;
            hs[o] = h;
            pitch[o] = (int)round_up(w, kPitchAlign);
            stride[o] = (int)round_up((int64_t)pitch[o] * h, 64);
            plane0[o] = off;
            off += (int64_t)stride[o] * kScales;
            c->geom[(size_t)i * kMaxOctaves + o] = OctGeom{plane0[o], w, h, pitch[o], stride[o]};
            w = (w + 1) / 2;
            h = (h + 1) / 2;
        }
        for (int o = 0; o < no; ++o) {
            OctJob j;
            memset(&j, 0, sizeof(j));
            j.plane0 = plane0[o];
            j.next0 = (o + 1 < no) ? plane0[o + 1] : -1;
            j.src = d.offset;
            j.w = ws[o];
            j.h = hs[o];
            j.pitch = pitch[o];
            j.plane_stride = stride[o];
            j.next_w = (o + 1 < no) ? ws[o + 1] : 0;
            j.next_h = (o + 1 < no) ? hs[o + 1] : 0;
            j.next_pitch = (o + 1 < no) ? pitch[o + 1] : 0;
            j.src_pitch = d.pitch;
            j.image = i;
            j.octave = o;
            for (int v = 0; v < kBlurTilings; ++v) j.tiles_x_blur[v] = (ws[o] + blur_tw(v) - 1) / blur_tw(v);
            per_oct[o].push_back(j);
        }
    }
    c->pyr_floats = off;
    c->jobs.clear();
    for (int o = 0; o < kMaxOctaves; ++o) {
        c->job_start[o] = (int)c->jobs.size();
        int tb[kBlurTilings] = {};
        for (OctJob& j : per_oct[o]) {
            for (int v = 0; v < kBlurTilings; ++v) {
                j.tile0_blur[v] = tb[v];
                tb[v] += j.tiles_x_blur[v] * ((j.h + blur_th(v) - 1) / blur_th(v));
            }
            c->jobs.push_back(j);
        }
        for (int v = 0; v < kBlurTilings; ++v) c->blur_tiles[v][o] = tb[v];
    }
    c->blur_owner.clear();
    for (int v = 0; v < kBlurTilings; ++v)
        for (int o = 0; o < kMaxOctaves; ++o) {
            c->blur_owner_start[v][o] = (int)c->blur_owner.size();
            for (size_t j = 0; j < per_oct[o].size(); ++j) {
                const OctJob& jb = per_oct[o][j];
                const int nt = jb.tiles_x_blur[v] * ((jb.h + blur_th(v) - 1) / blur_th(v));
                for (int t = 0; t < nt; ++t) c->blur_owner.push_back((int32_t)j);
            }
        }
    // BMLoG blocks: per octave, every job's grid of kBmStep-pixel block centres
    c->bm_blocks.clear();
    for (int o = 0; o < kMaxOctaves; ++o) {
        c->bm_start[o] = (int)(c->bm_blocks.size() / 3);
        for (size_t j = 0; j < per_oct[o].size(); ++j) {
            const OctJob& jb = per_oct[o][j];
            const int nbx = (jb.w + kBmStep - 1) / kBmStep, nby = (jb.h + kBmStep - 1) / kBmStep;
            for (int by = 0; by < nby; ++by)
                for (int bx = 0; bx < nbx; ++bx) {
                    c->bm_blocks.push_back((int32_t)j);
                    c->bm_blocks.push_back(bx);
                    c->bm_blocks.push_back(by);
                }
        }
        c->bm_count[o] = (int)(c->bm_blocks.size() / 3) - c->bm_start[o];
    }
    // candidate capacity per image: kCandCap, or one slot per 64 base pixels
    // for larger images (noise extrema of the first octave alone come to
    // about one per 200 pixels at the default contrast)
    c->cand_off.assign(c->n, 0);
    c->cand_cap.assign(c->n, 0);
    int64_t cand_total = 0;
    for (int i = 0; i < c->n; ++i) {
        const int64_t want = round_up((int64_t)c->images[i].width * c->images[i].height / 64, kCandBlock);
        c->cand_cap[i] = (int32_t)std::min<int64_t>(std::max<int64_t>(kCandCap, want), 1 << 24);
        c->cand_off[i] = cand_total;
        cand_total += c->cand_cap[i];
    }
    // strips of the ungated detection, covering each octave's centres inside
    // the border; image-major so that each XCD's contiguous share holds
    // whole images (balanced work, and neighbouring strips share halo rows
    // in that XCD's L2)
    c->strips.clear();
    for (int i = 0; i < c->n; ++i)
        for (int o = 0; o < kMaxOctaves; ++o)
            for (const OctJob& j : per_oct[o]) {
                if (j.image != i) continue;
                const int b = c->params.border;
                const int cw = j.w - 2 * b, ch = j.h - 2 * b;
                if (cw <= 0 || ch <= 0) continue;
                const int sx = (cw + kDetStripW - 1) / kDetStripW, sy = (ch + kDetStripH - 1) / kDetStripH;
                for (int t = 0; t < sx * sy; ++t) {
                    DetTile r;
                    memset(&r, 0, sizeof(r));
                    r.plane0 = j.plane0;
                    r.plane_stride = j.plane_stride;
                    r.pitch = j.pitch;
                    r.w = j.w;
                    r.h = j.h;
                    r.tx0 = b + (t % sx) * kDetStripW;
                    r.ty0 = b + (t / sx) * kDetStripH;
                    r.image = j.image;
                    r.octave = j.octave;
                    r.cand_cap = c->cand_cap[j.image];
                    r.cand_blk = (int32_t)(c->cand_off[j.image] / kCandBlock);
                    c->strips.push_back(r);
                }
            }
    c->job_start[kMaxOctaves] = (int)c->jobs.size();
    // surrogate CNN cells: 4x4-pixel cells of each base image
    c->cnn.assign(c->n, CnnImage{});
    int64_t cell = 0;
    int tiles = 0, chunks = 0, ftiles = 0;
    for (int i = 0; i < c->n; ++i) {
        const cdvs_image_desc& d = c->images[i];
        CnnImage& g = c->cnn[i];
        g.cell0 = cell;
        g.src = d.offset;
        g.src_pitch = d.pitch;
        g.H = d.height;
        g.W = d.width;
        g.H4 = (d.height + 3) / 4;
        g.W4 = (d.width + 3) / 4;
        g.n_oct = std::min(c->octaves[i], kCnnHeads);
        g.tiles_x = (g.W4 + kCnnTileW - 1) / kCnnTileW;
        g.tile0 = tiles;
        g.chunk0 = chunks;
        g.ftiles_x = (g.W4 + kCnnFusedW - 1) / kCnnFusedW;
        g.ftile0 = ftiles;
        ftiles += g.ftiles_x * ((g.H4 + kCnnFusedH - 1) / kCnnFusedH);
        c->cnn_owner.resize(ftiles, i);
        tiles += g.tiles_x * ((g.H4 + kCnnTileH - 1) / kCnnTileH);
        chunks += g.tiles_x * g.H4;
        cell += (int64_t)g.H4 * g.W4;
    }
    c->ncells = cell;
    c->cnn_tiles = tiles;
    c->cnn_chunks = chunks;
    c->cnn_ftiles = ftiles;
    return CDVS_OK;
}

// Largest power of two s such that a histogram bin of a window of radius
// `radius` (times the largest octave scale 2 sigma0) cannot exceed 2^32 - 1:
// a box side holds at most 2R + 1 pixels and one pixel adds at most
// |grad| <= 255 sqrt(2) < 361 to a bin (all weights are <= 1).
static float fixed_scale(double radius, double sigma0) {
    const double R = radius * 2.0 * sigma0;
    const double bound = (2.0 * R + 1.0) * (2.0 * R + 1.0) * 361.0;
    return (float)ldexp(1.0, (int)floor(log2(4294967295.0 / bound)));
}

static void build_constants(cdvs_ctx* c) {
    const cdvs_params& p = c->params;
    const double s0 = 1.6;
    const int radii[kScales] = {kR0, kR1, kR2, kR3, kR4};
    memset(&c->taps, 0, sizeof(c->taps));
    for (int k = 0; k < kScales; ++k) {
        const double s = (k == 0) ? s0 : s0 * sqrt(pow(2.0, k / 2.0) - 1.0);
        make_taps(s, radii[k], c->taps.g[k]);
    }
    // BMLoG transfer functions: the DFT over kBmN points of each tap set
    // (taps in double, normalised), real for symmetric taps; then the
    // products of the base blur's with each scale's
    {
        double Hd[kScales][kBmN];
        for (int k = 0; k < kScales; ++k) {
            const double sk = (k == 0) ? s0 : s0 * sqrt(pow(2.0, k / 2.0) - 1.0);
            const int r = radii[k];
            double t[2 * kMaxR + 1], sum = 0.0;
            for (int p = -r; p <= r; ++p) sum += (t[p + r] = exp(-(double)(p * p) / (2.0 * sk * sk)));
            for (int u = 0; u < kBmN; ++u) {
                double a = t[r] / sum;
                for (int p = 1; p <= r; ++p) a += 2.0 * t[r + p] / sum * cos(2.0 * M_PI * u * p / kBmN);
                Hd[k][u] = a;
            }
        }
        for (int u = 0; u < kBmN; ++u) {
            for (int k = 0; k < kScales; ++k) c->bm_H[k * kBmN + u] = (float)Hd[k][u];
            for (int k = 1; k < kScales; ++k) c->bm_H[(4 + k) * kBmN + u] = (float)(Hd[0][u] * Hd[k][u]);
        }
    }
    double sig[kScales];
    for (int k = 0; k < kScales; ++k) sig[k] = s0 * pow(2.0, k / 4.0);
    float beta[kScales][4];
    make_beta(sig, beta);
    for (int k = 0; k < kScales; ++k)
        for (int i = 0; i < 4; ++i) c->det.bsig[k][i] = (float)((double)beta[k][i] * sig[k] * sig[k]);
    c->det.lo = (float)sig[0];
    c->det.hi = (float)sig[kScales - 1];
    c->det.contrast = p.contrast;
    c->det.edge_lim = (p.edge_r + 1.f) * (p.edge_r + 1.f) / p.edge_r;
    c->det.max_off = p.max_offset;
    c->det.border = p.border;
    c->dedup_ratio = (float)pow(2.0, (double)p.dedup_dlog2);
    // the fixed-point scales are powers of two: their inverses and base-2
    // logarithms are exact
    const float ofix = fixed_scale(p.ori_radius, p.sigma0), dfix = fixed_scale(p.desc_radius, p.sigma0);
    const KpDiv kd = make_kp_div((uint32_t)c->kp_cap);
    c->ori = OriParams{p.ori_radius, p.ori_wsigma, p.ori_peak, p.sigma0, ofix, 1.f / ofix, (float)ilogb(ofix),
                       p.max_ori, c->kp_cap, kd};
    c->desc = DescParams{p.desc_cell, p.desc_radius, p.desc_wsigma, p.desc_clamp, p.sigma0,
                         dfix, 1.f / dfix, (float)ilogb(dfix), c->kp_cap, kd};
}

cdvs_status cdvs_ctx_create(const cdvs_params* params, const cdvs_image_desc* images, int32_t n_images,
                            int32_t kp_capacity, cdvs_ctx** out) {
    if (!out) return fail(nullptr, CDVS_ERR_ARG, "out is NULL");
    *out = nullptr;
    char msg[256];
    cdvs_status st = cdvs_validate(params, images, n_images, kp_capacity, msg, sizeof(msg));
    if (st != CDVS_OK) return fail(nullptr, st, "%s", msg);
    cdvs_ctx* c = new cdvs_ctx();
    c->params = *params;
    c->n = n_images;
    c->kp_cap = kp_capacity;
    c->images.assign(images, images + n_images);
    build_layout(c);
    build_constants(c);
    hipError_t e = hipSuccess;
    const size_t n = (size_t)n_images;
#define ALLOC(ptr, bytes)                                                        \
    do {                                                                         \
        e = hipMalloc((void**)&(ptr), (bytes));                                  \
        if (e != hipSuccess) {                                                   \
            fail(nullptr, CDVS_ERR_HIP, "hipMalloc(%zu): %s", (size_t)(bytes), hipGetErrorString(e)); \
            cdvs_ctx_destroy(c);                                                 \
            return CDVS_ERR_HIP;                                                 \
        }                                                                        \
    } while (0)
    ALLOC(c->d_jobs, sizeof(OctJob) * std::max<size_t>(1, c->jobs.size()));
    ALLOC(c->d_strips, sizeof(DetTile) * std::max<size_t>(1, c->strips.size()));
    ALLOC(c->d_blur_owner, sizeof(int32_t) * std::max<size_t>(1, c->blur_owner.size()));
    ALLOC(c->d_cnn_owner, sizeof(int32_t) * std::max<size_t>(1, c->cnn_owner.size()));
    ALLOC(c->d_geom, sizeof(OctGeom) * c->geom.size());
    {
        int64_t total = 0;
        int32_t cmax = 0;
        for (int i = 0; i < n; ++i) {
            total += c->cand_cap[i];
            cmax = std::max(cmax, c->cand_cap[i]);
        }
        ALLOC(c->d_cand, sizeof(cdvs_keypoint) * total);
        ALLOC(c->d_cand_off, sizeof(int64_t) * n);
        ALLOC(c->d_cand_capv, sizeof(int32_t) * n);
        if (cmax > kCandCap) ALLOC(c->d_sel, sizeof(cdvs_keypoint) * n * kCandCap);
    }
    ALLOC(c->d_cand_cnt, sizeof(int32_t) * (n + kXcds));
    ALLOC(c->d_ori, sizeof(cdvs_keypoint) * n * kp_capacity * kMaxOri);
    ALLOC(c->d_ori_cnt, sizeof(int32_t) * n * kp_capacity);
    ALLOC(c->d_flags, sizeof(int32_t));
    ALLOC(c->d_cnn, sizeof(CnnImage) * n);
    ALLOC(c->d_active, sizeof(int32_t) * n * kMaxOctaves);
    ALLOC(c->d_cnn_frag, sizeof(short) * kCnnFragShorts);
    ALLOC(c->d_scfv_prep, sizeof(float) * kScfvPrepFloats);
    ALLOC(c->d_wh, sizeof(int32_t) * 2 * n);
    ALLOC(c->d_img, sizeof(cdvs_image_desc) * n);
    ALLOC(c->d_bm_blocks, sizeof(int32_t) * std::max<size_t>(1, c->bm_blocks.size()));
    ALLOC(c->d_bm_H, sizeof(float) * kBmTransfers * kBmN);
#undef ALLOC
    std::vector<int32_t> wh(2 * n);
    for (size_t i = 0; i < n; ++i) {
        wh[2 * i] = images[i].width;
        wh[2 * i + 1] = images[i].height;
    }
    if ((e = hipMemcpy(c->d_jobs, c->jobs.data(), sizeof(OctJob) * c->jobs.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_strips, c->strips.data(), sizeof(DetTile) * c->strips.size(), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(c->d_blur_owner, c->blur_owner.data(), sizeof(int32_t) * c->blur_owner.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_cnn_owner, c->cnn_owner.data(), sizeof(int32_t) * c->cnn_owner.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_geom, c->geom.data(), sizeof(OctGeom) * c->geom.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_cnn, c->cnn.data(), sizeof(CnnImage) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_wh, wh.data(), sizeof(int32_t) * 2 * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_img, images, sizeof(cdvs_image_desc) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (!c->bm_blocks.empty() &&
         (e = hipMemcpy(c->d_bm_blocks, c->bm_blocks.data(), sizeof(int32_t) * c->bm_blocks.size(),
                        hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipMemcpy(c->d_bm_H, c->bm_H, sizeof(float) * kBmTransfers * kBmN, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(c->d_cand_off, c->cand_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_cand_capv, c->cand_cap.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemset(c->d_flags, 0, sizeof(int32_t))) != hipSuccess ||
        (e = hipMemset(c->d_cand_cnt, 0, sizeof(int32_t) * (n + kXcds))) != hipSuccess) {
        fail(nullptr, CDVS_ERR_HIP, "context upload: %s", hipGetErrorString(e));
        cdvs_ctx_destroy(c);
        return CDVS_ERR_HIP;
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    c->wgrad_grid = std::max(kXcds, cus * 2);
    // persistent detection: five 256-lane workgroups per compute unit (its
    // registers allow five waves per SIMD)
    c->detect_grid = std::max(kXcds, cus * 5 / kXcds * kXcds);
    *out = c;
    return CDVS_OK;
}

int64_t cdvs_pyramid_bytes(const cdvs_ctx* ctx) { return ctx ? ctx->pyr_floats * (int64_t)sizeof(float) : -1; }

int32_t cdvs_num_octaves(const cdvs_ctx* ctx, int32_t image) {
    if (!ctx || image < 0 || image >= ctx->n) return -1;
    return ctx->octaves[image];
}

int32_t cdvs_candidate_capacity(const cdvs_ctx* ctx) {
    if (!ctx) return -1;
    int32_t m = ctx->cand_cap.empty() ? kCandCap : ctx->cand_cap[0];
    for (int32_t v : ctx->cand_cap) m = std::min(m, v);
    return m;
}

cdvs_status cdvs_plane_layout(const cdvs_ctx* ctx, int32_t image, int32_t octave, int32_t k, int64_t* offset,
                              int32_t* width, int32_t* height, int32_t* pitch) {
    if (!ctx) return CDVS_ERR_STATE;
    if (image < 0 || image >= ctx->n || octave < 0 || octave >= ctx->octaves[image] || k < 0 || k >= kScales)
        return CDVS_ERR_ARG;
    const OctGeom& g = ctx->geom[(size_t)image * kMaxOctaves + octave];
    if (offset) *offset = g.plane0 + (int64_t)k * g.plane_stride;
    if (width) *width = g.w;
    if (height) *height = g.h;
    if (pitch) *pitch = g.pitch;
    return CDVS_OK;
}

cdvs_status cdvs_pyramid(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_images || !d_pyr) return fail(ctx, CDVS_ERR_ARG, "cdvs_pyramid: null device pointer");
    if (((uintptr_t)d_pyr & 255) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_pyramid: d_pyr not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    {
        Bracket b(ctx, CDVS_KERNEL_PREBLUR, s);
        HIP_OR_FAIL(ctx, launch_preblur(d_images, d_pyr, ctx->d_jobs + ctx->job_start[0],
                                        ctx->d_blur_owner + ctx->blur_owner_start[kPreblurVariant][0],
                                        ctx->blur_tiles[kPreblurVariant][0],
                                        ctx->taps, s));
    }
    for (int o = 0; o < ctx->max_oct; ++o) {
        Bracket b(ctx, CDVS_KERNEL_SCALES, s);
        const int v = ctx->blur_variant;
        HIP_OR_FAIL(ctx, launch_scales(d_pyr, ctx->d_jobs + ctx->job_start[o],
                                       ctx->d_blur_owner + ctx->blur_owner_start[v][o], ctx->blur_tiles[v][o], v,
                                       ctx->taps, s));
    }
    return CDVS_OK;
}

cdvs_status cdvs_pyramid_bmlog(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_images || !d_pyr) return fail(ctx, CDVS_ERR_ARG, "cdvs_pyramid_bmlog: null device pointer");
    if (((uintptr_t)d_pyr & 255) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_pyramid_bmlog: d_pyr not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    for (int o = 0; o < ctx->max_oct; ++o) {
        Bracket b(ctx, CDVS_KERNEL_BMLOG, s);
        HIP_OR_FAIL(ctx, launch_bmlog(d_images, d_pyr, ctx->d_jobs + ctx->job_start[o],
                                      ctx->d_bm_blocks + 3 * (int64_t)ctx->bm_start[o], ctx->bm_count[o],
                                      ctx->d_bm_H, o == 0, s));
    }
    return CDVS_OK;
}

cdvs_status cdvs_alp_detect(cdvs_ctx* ctx, const float* d_pyr, const uint8_t* d_mask, cdvs_keypoint* d_kp,
                            int32_t* d_count, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_pyr || !d_kp || !d_count) return fail(ctx, CDVS_ERR_ARG, "cdvs_alp_detect: null device pointer");
    if (((uintptr_t)d_pyr & 255) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_alp_detect: d_pyr not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    GateParams gate{nullptr, nullptr, nullptr, 1.f};
    if (d_mask) {
        Bracket b(ctx, CDVS_KERNEL_MASK_COUNT, s);
        HIP_OR_FAIL(ctx, launch_mask_count(d_mask, ctx->d_cnn, ctx->n, ctx->d_active, s));
        gate = GateParams{d_mask, ctx->d_active, ctx->d_cnn, ctx->params.mask_fmax};
    }
    {
        Bracket b(ctx, CDVS_KERNEL_CLEAR, s);
        HIP_OR_FAIL(ctx, launch_clear(ctx->d_cand_cnt, ctx->n + kXcds, s));   // counts and work counters
    }
    {
        // one launch over the strips of every octave; the finalisation does
        // not rely on the order in which candidates arrive
        Bracket b(ctx, CDVS_KERNEL_DETECT, s);
        HIP_OR_FAIL(ctx, launch_detect_strips(d_pyr, ctx->d_strips, (int)ctx->strips.size(), ctx->detect_variant,
                                              ctx->detect_grid, ctx->det, gate, ctx->d_cand_cnt + ctx->n,
                                              ctx->d_cand, ctx->d_cand_cnt, ctx->d_flags, s));
    }
    {
        Bracket b(ctx, CDVS_KERNEL_FINALIZE, s);
        HIP_OR_FAIL(ctx, launch_select(ctx->d_cand, ctx->d_cand_cnt, ctx->d_cand_off, ctx->d_cand_capv, ctx->n,
                                       ctx->d_sel, s));
        HIP_OR_FAIL(ctx, launch_finalize(ctx->d_cand, ctx->d_cand_cnt, ctx->d_cand_off, ctx->d_cand_capv, ctx->d_sel,
                                         ctx->n, ctx->dedup_ratio, ctx->params.topk, ctx->kp_cap, d_kp, d_count,
                                         ctx->d_flags, s));
    }
    return CDVS_OK;
}

cdvs_status cdvs_orient(cdvs_ctx* ctx, const float* d_pyr, const cdvs_keypoint* d_kp_in, const int32_t* d_count_in,
                        cdvs_keypoint* d_kp_out, int32_t* d_count_out, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_pyr || !d_kp_in || !d_count_in || !d_kp_out || !d_count_out)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_orient: null device pointer");
    if (((uintptr_t)d_pyr & 255) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_orient: d_pyr not 256-byte aligned");
    if ((const void*)d_kp_in == (const void*)d_kp_out || (const void*)d_count_in == (const void*)d_count_out)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_orient: outputs must not alias inputs");
    hipStream_t s = (hipStream_t)stream;
    {
        Bracket b(ctx, CDVS_KERNEL_ORIENT, s);
        HIP_OR_FAIL(ctx, launch_orient(d_pyr, ctx->d_geom, d_kp_in, d_count_in, ctx->n, ctx->ori, ctx->d_ori,
                                       ctx->d_ori_cnt, s));
    }
    {
        Bracket b(ctx, CDVS_KERNEL_ORIENT_COMPACT, s);
        HIP_OR_FAIL(ctx, launch_orient_compact(ctx->d_ori, ctx->d_ori_cnt, d_count_in, ctx->n, ctx->kp_cap,
                                               ctx->params.topk, d_kp_out, d_count_out, s));
    }
    return CDVS_OK;
}

cdvs_status cdvs_describe(cdvs_ctx* ctx, const float* d_pyr, const cdvs_keypoint* d_kp, const int32_t* d_count,
                          float* d_desc, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_pyr || !d_kp || !d_count || !d_desc) return fail(ctx, CDVS_ERR_ARG, "cdvs_describe: null device pointer");
    if (((uintptr_t)d_pyr & 255) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_describe: d_pyr not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    Bracket b(ctx, CDVS_KERNEL_DESCRIBE, s);
    HIP_OR_FAIL(ctx, launch_describe(d_pyr, ctx->d_geom, d_kp, d_count, ctx->n, ctx->desc, d_desc, s));
    return CDVS_OK;
}

cdvs_status cdvs_sync_status(cdvs_ctx* ctx, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    HIP_OR_FAIL(ctx, hipStreamSynchronize((hipStream_t)stream));
    int32_t flags = 0;
    HIP_OR_FAIL(ctx, hipMemcpy(&flags, ctx->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags) {
        HIP_OR_FAIL(ctx, hipMemset(ctx->d_flags, 0, sizeof(int32_t)));
        if (flags & kFlagFrontShape)
            return fail(ctx, CDVS_ERR_SHAPE,
                        "cdvs_front_end: a source image's size does not map onto the context's image of the "
                        "same index (or its descriptor is invalid); that image was not written");
        if (flags & kFlagCandOverflow)
            return fail(ctx, CDVS_ERR_CAPACITY,
                        "candidate scratch overflowed (an image found more candidates than its capacity, "
                        "max(%d, W*H/64)); results truncated", kCandCap);
        return fail(ctx, CDVS_ERR_CAPACITY,
                    "an image with more than %d candidates kept keypoints as weak as the weakest of its %d "
                    "strongest; its top-k may differ from the exact one", kCandCap, kCandCap);
    }
    return CDVS_OK;
}

static_assert(CDVS_SCFV_COMPONENTS == kScfvComponents && CDVS_SCFV_DIM == kScfvDim, "SCFV shape");

cdvs_status cdvs_scfv(cdvs_ctx* ctx, const cdvs_scfv_model* model, const float* d_desc, const int32_t* d_count,
                      float* d_gm, float* d_gv, float* d_delta, int32_t* d_order, uint32_t* d_bits, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!model || !model->d_pca_mean || !model->d_pca_matrix || !model->d_weights || !model->d_means ||
        !model->d_variances || !d_desc || !d_count || !d_gm || !d_gv || !d_delta || !d_order || !d_bits)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_scfv: null pointer");
    if ((((uintptr_t)d_desc | (uintptr_t)model->d_pca_mean) & 15) != 0)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_scfv: d_desc and the PCA mean must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    Bracket b(ctx, CDVS_KERNEL_SCFV, s);
    HIP_OR_FAIL(ctx, launch_scfv(d_desc, d_count, ctx->n, ctx->kp_cap, model->d_pca_mean, model->d_pca_matrix,
                                 model->d_weights, model->d_means, model->d_variances, ctx->d_scfv_prep, d_gm, d_gv,
                                 d_delta, d_order, d_bits, s));
    return CDVS_OK;
}

static_assert(CDVS_FRONT_LONG_SIDE == kFrontLongSide, "front-end long side");

cdvs_status cdvs_front_size(int32_t width, int32_t height, int32_t* out_width, int32_t* out_height) {
    if (!out_width || !out_height) return fail(nullptr, CDVS_ERR_ARG, "cdvs_front_size: null pointer");
    if (width < 1 || height < 1 || width > CDVS_MAX_SIDE || height > CDVS_MAX_SIDE)
        return fail(nullptr, CDVS_ERR_SHAPE, "cdvs_front_size: %d x %d outside 1..%d per side", width, height,
                    CDVS_MAX_SIDE);
    int w = 0, h = 0;
    front_size(width, height, &w, &h);
    *out_width = w;
    *out_height = h;
    return CDVS_OK;
}

cdvs_status cdvs_front_end(cdvs_ctx* ctx, const uint8_t* d_src, const cdvs_image_desc* d_src_desc,
                           uint8_t* d_images, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_src || !d_src_desc || !d_images) return fail(ctx, CDVS_ERR_ARG, "cdvs_front_end: null pointer");
    if ((const void*)d_src == (const void*)d_images)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_front_end: output must not alias the sources");
    hipStream_t s = (hipStream_t)stream;
    Bracket b(ctx, CDVS_KERNEL_FRONT, s);
    HIP_OR_FAIL(ctx, launch_front(d_src, d_src_desc, d_images, ctx->d_img, ctx->n, ctx->d_flags, s));
    return CDVS_OK;
}

static_assert(CDVS_SCFV_STATIC_BYTES == kScfvStaticFloats * 4, "static scratch size");

cdvs_status cdvs_scfv_noalloc(const cdvs_scfv_model* model, const float* d_desc, const int32_t* d_count,
                              int32_t n_images, int32_t kp_capacity, float* d_gm, float* d_gv, float* d_delta,
                              int32_t* d_order, uint32_t* d_bits, void* stream) {
    if (!model || !model->d_pca_mean || !model->d_pca_matrix || !model->d_weights || !model->d_means ||
        !model->d_variances || !d_desc || !d_count || !d_gm || !d_gv || !d_delta || !d_order || !d_bits)
        return fail(nullptr, CDVS_ERR_ARG, "cdvs_scfv_noalloc: null pointer");
    if (n_images < 0 || n_images > CDVS_MAX_IMAGES)
        return fail(nullptr, CDVS_ERR_ARG, "cdvs_scfv_noalloc: n_images %d outside 0..%d", n_images, CDVS_MAX_IMAGES);
    if (kp_capacity < 1 || kp_capacity > CDVS_MAX_KP_CAPACITY)
        return fail(nullptr, CDVS_ERR_ARG, "cdvs_scfv_noalloc: kp_capacity %d outside 1..%d (the maximum)",
                    kp_capacity, CDVS_MAX_KP_CAPACITY);
    if ((((uintptr_t)d_desc | (uintptr_t)model->d_pca_mean) & 15) != 0)
        return fail(nullptr, CDVS_ERR_ARG, "cdvs_scfv_noalloc: d_desc and the PCA mean must be 16-byte aligned");
    if (n_images == 0) return CDVS_OK;
    const int splits = scfv_static_splits(n_images, kp_capacity);
    if (splits > 1 && (int64_t)n_images * splits > kScfvStaticPartials)
        return fail(nullptr, CDVS_ERR_CAPACITY,
                    "cdvs_scfv_noalloc: %d images in %d parts need %lld partial blocks, the static scratch holds %d",
                    n_images, splits, (long long)n_images * splits, kScfvStaticPartials);
    float* scr = nullptr;
    hipError_t e = scfv_static_scratch(&scr);
    if (e != hipSuccess)
        return fail(nullptr, CDVS_ERR_HIP, "cdvs_scfv_noalloc: device address of the static scratch: %s",
                    hipGetErrorString(e));
    e = launch_scfv_static(scr, splits, d_desc, d_count, n_images, kp_capacity, model->d_pca_mean,
                           model->d_pca_matrix, model->d_weights, model->d_means, model->d_variances, d_gm, d_gv,
                           d_delta, d_order, d_bits, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, CDVS_ERR_HIP, "cdvs_scfv_noalloc: launch: %s", hipGetErrorString(e));
    return CDVS_OK;
}

static_assert(CDVS_REL_FEATURES == kRelFeatures && CDVS_REL_EDGES == kRelEdges && CDVS_REL_BINS == kRelBins,
              "relevance tables");

cdvs_status cdvs_relevance_select(cdvs_ctx* ctx, const cdvs_relevance_model* model, const cdvs_keypoint* d_kp_in,
                                  const int32_t* d_count_in, int32_t n_keep, cdvs_keypoint* d_kp_out,
                                  int32_t* d_count_out, float* d_score, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!model || !model->d_edges || !model->d_values || !d_kp_in || !d_count_in || !d_kp_out || !d_count_out)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_relevance_select: null pointer");
    if (n_keep < 1) return fail(ctx, CDVS_ERR_ARG, "cdvs_relevance_select: n_keep %d < 1", n_keep);
    if ((const void*)d_kp_in == (const void*)d_kp_out || (const void*)d_count_in == (const void*)d_count_out)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_relevance_select: outputs must not alias inputs");
    hipStream_t s = (hipStream_t)stream;
    Bracket b(ctx, CDVS_KERNEL_RELEVANCE, s);
    HIP_OR_FAIL(ctx, launch_relevance(d_kp_in, d_count_in, ctx->d_wh, ctx->n, ctx->kp_cap, model->d_edges,
                                      model->d_values, n_keep, d_kp_out, d_count_out, d_score, s));
    return CDVS_OK;
}

static_assert(CDVS_TQ_WORDS == kTqWords, "code words");

cdvs_status cdvs_encode(cdvs_ctx* ctx, const cdvs_tq_model* model, int32_t n_elements, const float* d_desc,
                        const int32_t* d_count, uint32_t* d_codes, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!model || !model->d_lo || !model->d_hi || !model->d_order || !d_desc || !d_count || !d_codes)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_encode: null pointer");
    if (n_elements < 1 || n_elements > kDescDim)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_encode: n_elements %d outside 1..%d", n_elements, kDescDim);
    if (((uintptr_t)d_desc & 15) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_encode: d_desc not 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    Bracket b(ctx, CDVS_KERNEL_ENCODE, s);
    HIP_OR_FAIL(ctx, launch_tq_encode(d_desc, d_count, ctx->n, ctx->kp_cap, model->d_lo, model->d_hi, model->d_order,
                                      n_elements, d_codes, s));
    return CDVS_OK;
}

int64_t cdvs_cnn_cells(const cdvs_ctx* ctx) { return ctx ? ctx->ncells : -1; }

cdvs_status cdvs_cnn_cell_layout(const cdvs_ctx* ctx, int32_t image, int64_t* cell0, int32_t* w4, int32_t* h4) {
    if (!ctx) return CDVS_ERR_STATE;
    if (image < 0 || image >= ctx->n) return CDVS_ERR_ARG;
    const CnnImage& g = ctx->cnn[image];
    if (cell0) *cell0 = g.cell0;
    if (w4) *w4 = g.W4;
    if (h4) *h4 = g.H4;
    return CDVS_OK;
}

cdvs_status cdvs_cnn_forward(cdvs_ctx* ctx, const uint8_t* d_images, const float* d_params, uint16_t* d_acts,
                             float* d_logits, uint8_t* d_mask, float tau, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_images || !d_params) return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_forward: null device pointer");
    if (d_mask && !(tau > 0.f && tau < 1.f)) return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_forward: tau must be in (0, 1)");
    if (((uintptr_t)d_acts & 7) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_forward: d_acts not 8-byte aligned");
    const float zthr = d_mask ? logf(tau / (1.f - tau)) : 0.f;
    hipStream_t s = (hipStream_t)stream;
    Bracket b(ctx, CDVS_KERNEL_CNN_FORWARD, s);
    if (!d_acts) {
        if (!d_logits && !d_mask) return CDVS_OK;
        HIP_OR_FAIL(ctx, launch_cnn_infer(d_images, d_params, ctx->d_cnn_frag, ctx->d_cnn, ctx->d_cnn_owner,
                                          ctx->cnn_ftiles, d_logits, d_mask, zthr, s));
        return CDVS_OK;
    }
    HIP_OR_FAIL(ctx, launch_cnn_forward(d_images, d_params, (short*)d_acts, ctx->ncells, ctx->d_cnn, ctx->n,
                                        ctx->cnn_tiles, d_logits, d_mask, zthr, s));
    return CDVS_OK;
}

cdvs_status cdvs_cnn_labels(cdvs_ctx* ctx, const cdvs_keypoint* d_kp, const int32_t* d_count, uint32_t* d_labels,
                            void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_kp || !d_count || !d_labels) return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_labels: null device pointer");
    HIP_OR_FAIL(ctx, launch_cnn_labels(d_kp, d_count, ctx->kp_cap, ctx->d_cnn, ctx->n, ctx->ncells, d_labels,
                                       (hipStream_t)stream));
    return CDVS_OK;
}

cdvs_status cdvs_cnn_backward(cdvs_ctx* ctx, const uint8_t* d_images, const float* d_params, const uint16_t* d_acts,
                              const float* d_logits, const uint32_t* d_labels, const float* d_pos_weight,
                              uint16_t* d_work, float* d_grad, float* d_loss, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_images || !d_params || !d_acts || !d_logits || !d_labels || !d_pos_weight || !d_work || !d_grad || !d_loss)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_backward: null device pointer");
    if ((((uintptr_t)d_acts | (uintptr_t)d_work) & 7) != 0)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_backward: d_acts and d_work must be 8-byte aligned");
    HIP_OR_FAIL(ctx, launch_cnn_backward(d_images, d_params, (const short*)d_acts, ctx->ncells, ctx->d_cnn, ctx->n,
                                         ctx->cnn_tiles, ctx->cnn_chunks, d_logits, d_labels, d_pos_weight,
                                         (short*)d_work, d_grad, d_loss, ctx->wgrad_grid, (hipStream_t)stream));
    return CDVS_OK;
}

cdvs_status cdvs_cnn_adam(cdvs_ctx* ctx, float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t step,
                          float lr, float beta1, float beta2, float eps, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_params || !d_grad || !d_m || !d_v) return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_adam: null device pointer");
    if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(ctx, CDVS_ERR_ARG, "cdvs_cnn_adam: bad hyper-parameters");
    HIP_OR_FAIL(ctx, launch_cnn_adam(d_params, d_grad, d_m, d_v, step, lr, beta1, beta2, eps, (hipStream_t)stream));
    return CDVS_OK;
}

// Records what `pass` enqueues on the context's capture stream into the
// context's graph, replacing any previous one.
static cdvs_status capture_into(cdvs_ctx* ctx, const std::function<cdvs_status(void*)>& pass) {
    if (!ctx->cap_stream) HIP_OR_FAIL(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    if (ctx->graph_exec) {
        (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
    }
    if (ctx->graph) {
        (void)hipGraphDestroy(ctx->graph);
        ctx->graph = nullptr;
    }
    HIP_OR_FAIL(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    const cdvs_status st = pass((void*)ctx->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (st != CDVS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(ctx, CDVS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    ctx->graph = g;
    HIP_OR_FAIL(ctx, hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0));
    return CDVS_OK;
}

cdvs_status cdvs_graph_capture(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, cdvs_keypoint* d_kp,
                               int32_t* d_count, cdvs_keypoint* d_kp_ori, int32_t* d_count_ori, float* d_desc) {
    if (!ctx) return CDVS_ERR_STATE;
    if (ctx->prof) return fail(ctx, CDVS_ERR_STATE, "cdvs_graph_capture: disable event timing first");
    if (!d_images || !d_pyr || !d_kp || !d_count || !d_kp_ori || !d_count_ori || !d_desc)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_graph_capture: null device pointer");
    return capture_into(ctx, [&](void* s) {
        cdvs_status st = cdvs_pyramid(ctx, d_images, d_pyr, s);
        if (st == CDVS_OK) st = cdvs_alp_detect(ctx, d_pyr, nullptr, d_kp, d_count, s);
        if (st == CDVS_OK) st = cdvs_orient(ctx, d_pyr, d_kp, d_count, d_kp_ori, d_count_ori, s);
        if (st == CDVS_OK) st = cdvs_describe(ctx, d_pyr, d_kp_ori, d_count_ori, d_desc, s);
        return st;
    });
}

cdvs_status cdvs_graph_capture_gated(cdvs_ctx* ctx, const uint8_t* d_images, const float* d_params, float tau,
                                     uint8_t* d_mask, float* d_pyr, cdvs_keypoint* d_kp, int32_t* d_count,
                                     cdvs_keypoint* d_kp_ori, int32_t* d_count_ori, float* d_desc) {
    if (!ctx) return CDVS_ERR_STATE;
    if (ctx->prof) return fail(ctx, CDVS_ERR_STATE, "cdvs_graph_capture_gated: disable event timing first");
    if (!d_images || !d_params || !d_mask || !d_pyr || !d_kp || !d_count || !d_kp_ori || !d_count_ori || !d_desc)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_graph_capture_gated: null device pointer");
    if (!(tau > 0.f && tau < 1.f)) return fail(ctx, CDVS_ERR_ARG, "cdvs_graph_capture_gated: tau must be in (0, 1)");
    return capture_into(ctx, [&](void* s) {
        cdvs_status st = cdvs_cnn_forward(ctx, d_images, d_params, nullptr, nullptr, d_mask, tau, s);
        if (st == CDVS_OK) st = cdvs_pyramid(ctx, d_images, d_pyr, s);
        if (st == CDVS_OK) st = cdvs_alp_detect(ctx, d_pyr, d_mask, d_kp, d_count, s);
        if (st == CDVS_OK) st = cdvs_orient(ctx, d_pyr, d_kp, d_count, d_kp_ori, d_count_ori, s);
        if (st == CDVS_OK) st = cdvs_describe(ctx, d_pyr, d_kp_ori, d_count_ori, d_desc, s);
        return st;
    });
}

cdvs_status cdvs_graph_launch(cdvs_ctx* ctx, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!ctx->graph_exec) return fail(ctx, CDVS_ERR_STATE, "cdvs_graph_launch: no captured graph");
    HIP_OR_FAIL(ctx, hipGraphLaunch(ctx->graph_exec, (hipStream_t)stream));
    return CDVS_OK;
}

int32_t cdvs_tune_get(const cdvs_ctx* ctx, int32_t kernel) {
    if (!ctx) return -1;
    if (kernel == CDVS_KERNEL_SCALES) return ctx->blur_variant;
    if (kernel == CDVS_KERNEL_DETECT) return ctx->detect_variant;
    return -1;
}
cdvs_status cdvs_tune_set(cdvs_ctx* ctx, int32_t kernel, int32_t variant) {
    if (!ctx) return CDVS_ERR_STATE;
    if (kernel == CDVS_KERNEL_SCALES) {
        if (variant < 0 || variant >= kBlurVariants)
            return fail(ctx, CDVS_ERR_ARG, "cdvs_tune_set: variant out of range");
        ctx->blur_variant = variant;
        return CDVS_OK;
    }
    if (kernel == CDVS_KERNEL_DETECT) {
        if (variant < 0 || variant >= kDetectVariants)
            return fail(ctx, CDVS_ERR_ARG, "cdvs_tune_set: variant out of range");
        ctx->detect_variant = variant;
        return CDVS_OK;
    }
    return fail(ctx, CDVS_ERR_ARG, "cdvs_tune_set: only CDVS_KERNEL_SCALES and CDVS_KERNEL_DETECT are tunable");
}

// Cache key: arch, size of the first image, batch size rounded up to a power of two.
static_assert(CDVS_TUNE_VARIANTS == kBlurVariants && CDVS_DETECT_VARIANTS == kDetectVariants,
              "tunable variant counts agree with the header");

static std::string tune_key(const cdvs_ctx* ctx) {
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    }
    int nb = 1;
    while (nb < ctx->n) nb <<= 1;
    char buf[160];
    snprintf(buf, sizeof(buf), "%s:pass:%dx%d:n%d", arch.c_str(), ctx->images[0].width, ctx->images[0].height, nb);
    return buf;
}

// The cache is a JSON object with one "key": {...} entry per line.
static bool tune_cache_lookup(const char* path, const std::string& key, int* variant, int* dvariant) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line, pat = "\"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(pat) == std::string::npos) continue;
        const size_t p = line.find("\"variant\":"), d = line.find("\"detect\":");
        if (p == std::string::npos || d == std::string::npos) return false;
        const int v = atoi(line.c_str() + p + 10), dv = atoi(line.c_str() + d + 9);
        if (v < 0 || v >= kBlurVariants || dv < 0 || dv >= kDetectVariants) return false;
        *variant = v;
        *dvariant = dv;
        return true;
    }
    return false;
}

static void tune_cache_store(const char* path, const std::string& key, int variant, const float* us, int dvariant,
                             const float* dus) {
    std::vector<std::string> entries;
    std::ifstream f(path);
    std::string line, pat = "\"" + key + "\"";
    while (f && std::getline(f, line)) {
        size_t q = line.find('"');
        if (q == std::string::npos || line.find(pat) != std::string::npos) continue;
        // keep only well-formed entries of other keys; anything else is dropped
        if (line.find("\"variant\": ") == std::string::npos || line.find("\"us\": [") == std::string::npos ||
            line.find("\"detect\": ") == std::string::npos)
            continue;
        size_t e = line.find_last_of('}');
        if (e == std::string::npos) continue;
        entries.push_back(line.substr(q, e - q + 1));
    }
    char buf[640];
    snprintf(buf, sizeof(buf),
             "\"%s\": {\"variant\": %d, \"us\": [%.1f, %.1f, %.1f, %.1f], \"detect\": %d, \"detect_us\": [%.1f, %.1f]}",
             key.c_str(), variant, us[0], us[1], us[2], us[3], dvariant, dus[0], dus[1]);
    entries.push_back(buf);
    std::ofstream o(path, std::ios::trunc);
    o << "{\n";
    for (size_t i = 0; i < entries.size(); ++i) o << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
    o << "}\n";
}

cdvs_status cdvs_autotune(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, const char* cache_path, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!d_images || !d_pyr) return fail(ctx, CDVS_ERR_ARG, "cdvs_autotune: null device pointer");
    if (((uintptr_t)d_pyr & 255) != 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_autotune: d_pyr not 256-byte aligned");
    const std::string key = tune_key(ctx);
    int v = 0, dv = 0;
    if (cache_path && tune_cache_lookup(cache_path, key, &v, &dv)) {
        ctx->blur_variant = v;
        ctx->detect_variant = dv;
        return CDVS_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_OR_FAIL(ctx, hipEventCreate(&e0));
    HIP_OR_FAIL(ctx, hipEventCreate(&e1));
    const bool prof = ctx->prof;
    ctx->prof = false;
    // Each variant is warmed up twice, then timed seven times with the
    // variants taken in turn inside each round, so a clock that is still
    // settling favours none of them; the median of each is kept.  Shapes can
    // be within 10% of each other, closer than a few samples separate.
    constexpr int kRuns = 7;
    auto time_variants = [&](int nvar, auto&& run, float* out) -> cdvs_status {
        std::vector<float> t((size_t)nvar * kRuns, 0.f);
        cdvs_status st = CDVS_OK;
        for (int w = 0; w < 2 && st == CDVS_OK; ++w)
            for (int var = 0; var < nvar && st == CDVS_OK; ++var) st = run(var);
        for (int r = 0; r < kRuns && st == CDVS_OK; ++r)
            for (int var = 0; var < nvar && st == CDVS_OK; ++var) {
                (void)hipEventRecord(e0, s);
                st = run(var);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                t[(size_t)var * kRuns + r] = ms * 1e3f;
            }
        for (int var = 0; var < nvar; ++var) {
            float* tv = t.data() + (size_t)var * kRuns;
            std::sort(tv, tv + kRuns);
            out[var] = tv[kRuns / 2];
        }
        return st;
    };
    auto argmin = [](const float* x, int n) {
        int b = 0;
        for (int i = 1; i < n; ++i)
            if (x[i] < x[b]) b = i;
        return b;
    };
    float us[kBlurVariants] = {}, dus[kDetectVariants] = {};
    int best_v = ctx->blur_variant, best_dv = ctx->detect_variant;
    cdvs_status st = time_variants(
        kBlurVariants,
        [&](int var) {
            ctx->blur_variant = var;
            return cdvs_pyramid(ctx, d_images, d_pyr, stream);
        },
        us);
    if (st == CDVS_OK) {
        best_v = argmin(us, kBlurVariants);
        // the detection's launch forms on the pyramid just built (every tile
        // shape writes the same planes), candidates into the context's scratch
        st = time_variants(
            kDetectVariants,
            [&](int var) -> cdvs_status {
                const GateParams gate{nullptr, nullptr, nullptr, 1.f};
                HIP_OR_FAIL(ctx, launch_clear(ctx->d_cand_cnt, ctx->n + kXcds, s));
                HIP_OR_FAIL(ctx, launch_detect_strips(d_pyr, ctx->d_strips, (int)ctx->strips.size(), var,
                                                      ctx->detect_grid, ctx->det, gate, ctx->d_cand_cnt + ctx->n,
                                                      ctx->d_cand, ctx->d_cand_cnt, ctx->d_flags, s));
                return CDVS_OK;
            },
            dus);
        if (st == CDVS_OK) best_dv = argmin(dus, kDetectVariants);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->prof = prof;
    ctx->blur_variant = best_v;
    ctx->detect_variant = best_dv;
    if (st != CDVS_OK) return st;
    if (cache_path) tune_cache_store(cache_path, key, best_v, us, best_dv, dus);
    return CDVS_OK;
}

cdvs_status cdvs_profile_enable(cdvs_ctx* ctx, int32_t enable) {
    if (!ctx) return CDVS_ERR_STATE;
    if (enable && ctx->ev.empty()) {
        ctx->ev.resize(2 * kMaxBrackets);
        ctx->ev_id.resize(kMaxBrackets);
        for (auto& e : ctx->ev) HIP_OR_FAIL(ctx, hipEventCreate(&e));
    }
    ctx->prof = enable != 0;
    return CDVS_OK;
}

cdvs_status cdvs_profile_read(cdvs_ctx* ctx, double* total_ms, int32_t* launches) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!total_ms || !launches) return fail(ctx, CDVS_ERR_ARG, "cdvs_profile_read: null output");
    for (int i = 0; i < CDVS_KERNEL_COUNT; ++i) {
        total_ms[i] = 0.0;
        launches[i] = 0;
    }
    if (ctx->ev_used > 0) HIP_OR_FAIL(ctx, hipEventSynchronize(ctx->ev[2 * ctx->ev_used - 1]));
    for (int b = 0; b < ctx->ev_used; ++b) {
        float ms = 0.f;
        HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, ctx->ev[2 * b], ctx->ev[2 * b + 1]));
        total_ms[ctx->ev_id[b]] += ms;
        launches[ctx->ev_id[b]] += 1;
    }
    ctx->ev_used = 0;
    return CDVS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Streaming with the host hand-off overlapped.

namespace {

// Hands chunk indices to the host thread and counts what it has finished.
struct ConsumerQueue {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int> q;
    int consumed = 0;     // chunks 0..consumed-1 are done
    bool closed = false;  // no more chunks
    bool failed = false;
    int fail_chunk = -1, fail_rc = 0;
    std::string fail_msg;
};

}  // namespace

static int64_t images_extent(const cdvs_ctx* ctx) {
    int64_t e = 0;
    for (const auto& d : ctx->images) e = std::max(e, d.offset + (int64_t)d.pitch * d.height);
    return e;
}

static void consumer_loop(ConsumerQueue* cq, const cdvs_stream_buffers* buf, hipEvent_t* copied,
                          cdvs_chunk_consumer consumer, void* user, int n, int cap) {
    for (;;) {
        int c;
        {
            std::unique_lock<std::mutex> lk(cq->mu);
            cq->cv.wait(lk, [&] { return !cq->q.empty() || cq->closed; });
            if (cq->q.empty()) return;
            c = cq->q.front();
            cq->q.pop_front();
        }
        const int slot = c & 1;
        hipError_t e = hipEventSynchronize(copied[slot]);
        int32_t rc = 0;
        bool skip;
        {
            std::lock_guard<std::mutex> lk(cq->mu);
            skip = cq->failed;
        }
        if (e == hipSuccess && !skip) rc = consumer(user, c, n, cap, buf->h_count[slot], buf->h_kp[slot], buf->h_desc[slot]);
        std::lock_guard<std::mutex> lk(cq->mu);
        if (e != hipSuccess || rc != 0) {
            if (!cq->failed) {
                cq->failed = true;
                cq->fail_chunk = c;
                cq->fail_rc = rc;
                cq->fail_msg = e != hipSuccess ? hipGetErrorString(e) : "";
            }
        }
        cq->consumed = c + 1;
        cq->cv.notify_all();
    }
}

extern "C" {

cdvs_status cdvs_stream(cdvs_ctx* ctx, const uint8_t* d_images, int64_t chunk_stride, int32_t n_chunks,
                        const cdvs_stream_buffers* buf, cdvs_chunk_consumer consumer, void* user, void* stream) {
    if (!ctx) return CDVS_ERR_STATE;
    if (!buf || !consumer || !d_images) return fail(ctx, CDVS_ERR_ARG, "cdvs_stream: null argument");
    if (!buf->d_pyr || !buf->d_kp || !buf->d_count || !buf->d_kp_ori || !buf->d_count_ori || !buf->d_desc)
        return fail(ctx, CDVS_ERR_ARG, "cdvs_stream: null device buffer");
    for (int sl = 0; sl < 2; ++sl)
        if (!buf->h_count[sl] || !buf->h_kp[sl] || !buf->h_desc[sl])
            return fail(ctx, CDVS_ERR_ARG, "cdvs_stream: null host slot %d", sl);
    const bool gated = buf->d_cnn_params != nullptr;
    if (gated && (!buf->d_mask || !(buf->tau > 0.f && buf->tau < 1.f)))
        return fail(ctx, CDVS_ERR_ARG, "cdvs_stream: gating needs d_mask and tau in (0, 1)");
    if (n_chunks < 0) return fail(ctx, CDVS_ERR_ARG, "cdvs_stream: n_chunks < 0");
    if (n_chunks > 1 && chunk_stride < images_extent(ctx))
        return fail(ctx, CDVS_ERR_ARG, "cdvs_stream: chunk_stride %lld below the batch extent %lld",
                    (long long)chunk_stride, (long long)images_extent(ctx));
    if (n_chunks == 0) return CDVS_OK;

    const int n = ctx->n, cap = ctx->kp_cap;
    hipStream_t s = (hipStream_t)stream, cs = nullptr;
    hipEvent_t done[2] = {}, copied[2] = {};
    HIP_OR_FAIL(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    cdvs_status st = CDVS_OK;
    for (int i = 0; i < 2 && st == CDVS_OK; ++i) {
        if (hipEventCreateWithFlags(&done[i], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&copied[i], hipEventDisableTiming) != hipSuccess)
            st = fail(ctx, CDVS_ERR_HIP, "cdvs_stream: hipEventCreate failed");
    }
    ConsumerQueue cq;
    std::thread host;
    if (st == CDVS_OK) host = std::thread(consumer_loop, &cq, buf, copied, consumer, user, n, cap);

    auto enq = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && st == CDVS_OK) st = fail(ctx, CDVS_ERR_HIP, "cdvs_stream: %s: %s", what, hipGetErrorString(e));
    };
    for (int c = 0; c < n_chunks && st == CDVS_OK; ++c) {
        const uint8_t* imgs = d_images + (int64_t)c * chunk_stride;
        const int slot = c & 1;
        st = cdvs_pyramid(ctx, imgs, buf->d_pyr, s);
        if (st == CDVS_OK && gated)
            st = cdvs_cnn_forward(ctx, imgs, buf->d_cnn_params, buf->d_acts, nullptr, buf->d_mask, buf->tau, s);
        if (st == CDVS_OK) st = cdvs_alp_detect(ctx, buf->d_pyr, gated ? buf->d_mask : nullptr, buf->d_kp, buf->d_count, s);
        // the oriented keypoints and descriptors of chunk c-1 must have left the device
        if (st == CDVS_OK && c > 0) enq(hipStreamWaitEvent(s, copied[slot ^ 1], 0), "wait for copy");
        if (st == CDVS_OK) st = cdvs_orient(ctx, buf->d_pyr, buf->d_kp, buf->d_count, buf->d_kp_ori, buf->d_count_ori, s);
        if (st == CDVS_OK) st = cdvs_describe(ctx, buf->d_pyr, buf->d_kp_ori, buf->d_count_ori, buf->d_desc, s);
        if (st == CDVS_OK) enq(hipEventRecord(done[slot], s), "record");
        if (st != CDVS_OK) break;
        {   // host slot `slot` last held chunk c-2: wait until it has been consumed
            std::unique_lock<std::mutex> lk(cq.mu);
            cq.cv.wait(lk, [&] { return cq.consumed >= c - 1 || cq.failed; });
            if (cq.failed) break;
        }
        enq(hipStreamWaitEvent(cs, done[slot], 0), "copy wait");
        enq(hipMemcpyAsync(buf->h_count[slot], buf->d_count_ori, sizeof(int32_t) * n, hipMemcpyDeviceToHost, cs), "D2H");
        enq(hipMemcpyAsync(buf->h_kp[slot], buf->d_kp_ori, sizeof(cdvs_keypoint) * n * cap, hipMemcpyDeviceToHost, cs),
            "D2H");
        enq(hipMemcpyAsync(buf->h_desc[slot], buf->d_desc, sizeof(float) * 128 * (int64_t)n * cap, hipMemcpyDeviceToHost,
                           cs), "D2H");
        enq(hipEventRecord(copied[slot], cs), "record");
        if (st != CDVS_OK) break;
        std::lock_guard<std::mutex> lk(cq.mu);
        cq.q.push_back(c);
        cq.cv.notify_all();
    }
    if (host.joinable()) {
        {
            std::lock_guard<std::mutex> lk(cq.mu);
            cq.closed = true;
            cq.cv.notify_all();
        }
        host.join();
    }
    // nothing may still be in flight into the caller's buffers when we return
    (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(cs);
    for (int i = 0; i < 2; ++i) {
        if (done[i]) (void)hipEventDestroy(done[i]);
        if (copied[i]) (void)hipEventDestroy(copied[i]);
    }
    (void)hipStreamDestroy(cs);
    if (st != CDVS_OK) return st;
    if (cq.failed) {
        if (!cq.fail_msg.empty())
            return fail(ctx, CDVS_ERR_HIP, "cdvs_stream: chunk %d copy: %s", cq.fail_chunk, cq.fail_msg.c_str());
        return fail(ctx, CDVS_ERR_STATE, "cdvs_stream: consumer returned %d for chunk %d", cq.fail_rc, cq.fail_chunk);
    }
    return cdvs_sync_status(ctx, stream);
}

int32_t cdvs_standin_consume(void* user, int32_t chunk, int32_t n_images, int32_t kp_capacity, const int32_t* h_count,
                             const cdvs_keypoint* h_kp, const float* h_desc) {
    (void)h_kp;
    const cdvs_standin_sink* sk = (const cdvs_standin_sink*)user;
    if (!sk || !sk->out || !sk->kept || !h_count || !h_desc || n_images < 0 || kp_capacity < 1) return 1;
    const int64_t first = (int64_t)chunk * n_images;
    if (chunk < 0 || first + n_images > sk->total_images) return 2;
    const int nt = std::max(1, std::min(sk->threads, std::max(1, n_images)));
    auto work = [&](int t) {
        for (int i = t; i < n_images; i += nt) {
            const int m = std::max(0, std::min({h_count[i], sk->keep, kp_capacity}));
            const float* src = h_desc + (int64_t)i * kp_capacity * 128;
            uint8_t* dst = sk->out + (first + i) * kp_capacity * 128;
            for (int64_t j = 0; j < (int64_t)m * 128; ++j) {
                const float q = floorf(src[j] * 512.f + 0.5f);
                dst[j] = (uint8_t)(q >= 255.f ? 255 : (q <= 0.f ? 0 : (int)q));
            }
            sk->kept[first + i] = m;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();
    return 0;
}

}  // extern "C"
