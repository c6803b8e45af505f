/*
 * CDVS front-half ORACLE -- test infrastructure, not product code.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  The GPU path never calls it, and it shares no code,
 * header, table or constant generator with the GPU path: every constant below
 * (Gaussian taps, the ALP least-squares matrix, octave sizes) is derived here
 * from the definitions, independently of the HIP library.
 *
 * It is a plain, slow, single-threaded transcription of what the method
 * computes, following "Fast MPEG-CDVS Encoder with GPU-CPU Hybrid Computing"
 * (Duan et al.), in the order the paper gives:
 *   - Sec. III-A, Eq. (1): Gaussian scale space by separable filters, then a
 *     3x3 Laplacian, scale-normalised (times sigma^2).
 *   - Sec. III-A, Eqs. (2)-(3): the ALP cubic in sigma per pixel, its
 *     extremal scale from p'(sigma) = 0, then the 8-neighbour comparison.
 *   - Sec. IV-A, Algorithm 1: per octave, stage A (filtering + ALP test),
 *     stage B (refine candidate position, drop unstable ones), stage C
 *     (compare candidates of adjacent octaves, the lower response loses),
 *     then downsample G_{o,4} to G_{o+1,0}.
 *   - Sec. III-B / IV-B, Algorithm 2: 36-bin orientation histogram within
 *     radius 3.96 sigma, orientations above 0.8 x the highest peak; the
 *     4x4-cell x 8-bin descriptor with cells 3 sigma wide within 6 sigma.
 * Where the paper is silent (pre-blur of the input, kernel radius, border,
 * Laplacian stencil, root choice, refinement and deduplication rules,
 * histogram weighting and interpolation, normalisation) the reading used is
 * the one listed in the design notes; weighting and normalisation follow
 * Lowe, "Distinctive image features from scale-invariant keypoints", IJCV 2004.
 *
 * Precision: REAL is double (the reference build, used for the mathematical
 * pins) or float (the build whose decisions -- thresholds, strict NMS, disk
 * membership, peak tests -- are taken in the same precision as the GPU
 * kernels).  Built with -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef REAL
#define REAL double
#endif
typedef REAL real;

#define IS_F32 (sizeof(real) == 4)
static real r_exp(real v) { return IS_F32 ? (real)expf((float)v) : (real)exp((double)v); }
static real r_sqrt(real v) { return IS_F32 ? (real)sqrtf((float)v) : (real)sqrt((double)v); }
static real r_atan2(real y, real x) {
    return IS_F32 ? (real)atan2f((float)y, (float)x) : (real)atan2((double)y, (double)x);
}
static real r_log2(real v) { return IS_F32 ? (real)log2f((float)v) : (real)log2((double)v); }
static real r_floor(real v) { return IS_F32 ? (real)floorf((float)v) : (real)floor((double)v); }
static real r_abs(real v) { return v < 0 ? -v : v; }

#define TWO_PI 6.283185307179586476925286766559

/* ---------------------------------------------------------------------- */
/* Parameters and records (the oracle's own types)                          */
/* ---------------------------------------------------------------------- */
typedef struct {
    double sigma0;      /* base scale of every octave */
    int32_t intervals;  /* S: scale images k = 0..S per octave */
    int32_t min_side;   /* stop after the first octave whose short side is below this */
    double contrast;    /* T: minimum |p| of a candidate */
    double edge_r;      /* edge ratio r: reject when tr^2/det >= (r+1)^2/r */
    int32_t border;     /* detection margin in octave pixels */
    int32_t ori_bins;   /* 36 */
    double max_offset;  /* refinement offset limit per axis (octave px) */
    double dedup_dlog2; /* stage C: |log2 sigma_a/sigma_b| limit */
    double ori_radius;  /* 3.96 (x sigma) */
    double ori_wsigma;  /* Gaussian weight sigma of the orientation window (x sigma) */
    double ori_peak;    /* 0.8 */
    int32_t max_ori;    /* at most this many orientations per keypoint */
    int32_t topk;       /* keypoints kept per image (<= 0: all) */
    double desc_cell;   /* cell side (x sigma) */
    double desc_radius; /* descriptor window radius (x sigma) */
    double desc_wsigma; /* descriptor Gaussian weight sigma (x sigma) */
    double desc_clamp;  /* clamp after the first normalisation */
} or_params;

typedef struct {
    double x, y, sigma, p;     /* base-image px; sigma in base px; p = response */
    double theta, rho, pss, peak;
    int32_t image, octave, ix, iy;
} or_kp;

void or_default_params(or_params* P) {
    P->sigma0 = 1.6;
    P->intervals = 4;
    P->min_side = 32;
    P->contrast = 1.5;
    P->edge_r = 10.0;
    P->border = 4;
    P->ori_bins = 36;
    P->max_offset = 0.5;
    P->dedup_dlog2 = 0.25;
    P->ori_radius = 3.96;
    P->ori_wsigma = 1.5;
    P->ori_peak = 0.8;
    P->max_ori = 4;
    P->topk = 1000;
    P->desc_cell = 3.0;
    P->desc_radius = 6.0;
    P->desc_wsigma = 6.0;
    P->desc_clamp = 0.2;
}

int or_real_size(void) { return (int)sizeof(real); }

/* ---------------------------------------------------------------------- */
/* Octave geometry (Algorithm 1: octaves by downsampling)                   */
/* ---------------------------------------------------------------------- */
/* Octave o has size ceil(W / 2^o) x ceil(H / 2^o).  Octaves are added while
 * the current one's short side is at least min_side; the first octave with a
 * short side below min_side is the last one. */
int or_num_octaves(int W, int H, int min_side) {
    int n = 1, w = W, h = H;
    while ((w < h ? w : h) >= min_side) {
        w = (w + 1) / 2;
        h = (h + 1) / 2;
        ++n;
    }
    return n;
}

void or_octave_size(int W, int H, int o, int* w, int* h) {
    int a = W, b = H;
    for (int i = 0; i < o; ++i) {
        a = (a + 1) / 2;
        b = (b + 1) / 2;
    }
    *w = a;
    *h = b;
}

/* Number of reals in the whole pyramid: per octave, S+1 planes of w_o*h_o. */
int64_t or_pyramid_len(int W, int H, const or_params* P) {
    int n = or_num_octaves(W, H, P->min_side);
    int64_t tot = 0;
    for (int o = 0; o < n; ++o) {
        int w, h;
        or_octave_size(W, H, o, &w, &h);
        tot += (int64_t)(P->intervals + 1) * w * h;
    }
    return tot;
}

/* Offset (in reals) of plane k of octave o. */
int64_t or_plane_offset(int W, int H, const or_params* P, int o, int k) {
    int64_t off = 0;
    for (int i = 0; i < o; ++i) {
        int w, h;
        or_octave_size(W, H, i, &w, &h);
        off += (int64_t)(P->intervals + 1) * w * h;
    }
    int w, h;
    or_octave_size(W, H, o, &w, &h);
    return off + (int64_t)k * w * h;
}

/* ---------------------------------------------------------------------- */
/* Gaussian filters (Eq. (1); Algorithm 1 stage A)                          */
/* ---------------------------------------------------------------------- */
/* Scale of image k of an octave, in octave pixels: sigma0 * 2^(k/S). */
double or_scale_sigma(const or_params* P, int k) {
    return P->sigma0 * pow(2.0, (double)k / (double)P->intervals);
}

/* Every G_{o,k} (k >= 1) is filtered directly from G_{o,0} (Algorithm 1 filters
 * G_{o,0} by g_k), so g_k must add sigma_k^2 - sigma0^2 of variance:
 * s_k = sigma0 * sqrt(2^(2k/S) - 1).  k = 0 is the pre-blur of the input,
 * which is taken as sharp, with s = sigma0. */
double or_blur_sigma(const or_params* P, int k) {
    if (k == 0) return P->sigma0;
    return P->sigma0 * sqrt(pow(2.0, 2.0 * k / (double)P->intervals) - 1.0);
}

int or_blur_radius(double s) { return (int)ceil(4.0 * s); }

/* Sampled Gaussian exp(-p^2 / (2 s^2)), |p| <= r, normalised to sum 1 in
 * double, then rounded to REAL.  taps has 2r+1 entries, taps[r] is p = 0. */
void or_gauss_taps(double s, int r, real* taps) {
    double sum = 0.0;
    for (int p = -r; p <= r; ++p) sum += exp(-(double)p * p / (2.0 * s * s));
    for (int p = -r; p <= r; ++p) taps[p + r] = (real)(exp(-(double)p * p / (2.0 * s * s)) / sum);
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Separable Gaussian, vertical pass first then horizontal (Algorithm 1 stage
 * A: T_k from a column sum over G_{o,0}, then G_{o,k} from a row sum over
 * T_k), taps summed in order p = -r..r, clamp-to-edge border. */
int or_blur(const real* in, int w, int h, double s, int r, real* out) {
    real* taps = (real*)malloc(sizeof(real) * (2 * r + 1));
    real* tmp = (real*)malloc(sizeof(real) * (size_t)w * h);
    if (!taps || !tmp) {
        free(taps);
        free(tmp);
        return -1;
    }
    or_gauss_taps(s, r, taps);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            real acc = 0;
            for (int p = -r; p <= r; ++p) acc += taps[p + r] * in[(size_t)clampi(y + p, 0, h - 1) * w + x];
            tmp[(size_t)y * w + x] = acc;
        }
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            real acc = 0;
            for (int p = -r; p <= r; ++p) acc += taps[p + r] * tmp[(size_t)y * w + clampi(x + p, 0, w - 1)];
            out[(size_t)y * w + x] = acc;
        }
    free(taps);
    free(tmp);
    return 0;
}

/* The whole pyramid (Algorithm 1 stage A and its last step).  The u8 input is
 * converted to 0..255 reals and pre-blurred by sigma0 to give G_{0,0}; each
 * octave's G_{o,k}, k = 1..S, is filtered from G_{o,0}; G_{o+1,0} takes the
 * even samples of G_{o,S}: G_{o+1,0}[i][j] = G_{o,S}[2i][2j]. */
int or_pyramid(const uint8_t* img, int W, int H, int pitch, const or_params* P, real* pyr) {
    int n = or_num_octaves(W, H, P->min_side);
    int S = P->intervals;
    real* base = (real*)malloc(sizeof(real) * (size_t)W * H);
    if (!base) return -1;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) base[(size_t)y * W + x] = (real)img[(size_t)y * pitch + x];
    int rc = or_blur(base, W, H, or_blur_sigma(P, 0), or_blur_radius(or_blur_sigma(P, 0)),
                     pyr + or_plane_offset(W, H, P, 0, 0));
    free(base);
    if (rc) return rc;
    for (int o = 0; o < n; ++o) {
        int w, h;
        or_octave_size(W, H, o, &w, &h);
        const real* g0 = pyr + or_plane_offset(W, H, P, o, 0);
        for (int k = 1; k <= S; ++k) {
            double s = or_blur_sigma(P, k);
            rc = or_blur(g0, w, h, s, or_blur_radius(s), pyr + or_plane_offset(W, H, P, o, k));
            if (rc) return rc;
        }
        if (o + 1 < n) {
            int w2, h2;
            or_octave_size(W, H, o + 1, &w2, &h2);
            const real* gs = pyr + or_plane_offset(W, H, P, o, S);
            real* nb = pyr + or_plane_offset(W, H, P, o + 1, 0);
            for (int i = 0; i < h2; ++i)
                for (int j = 0; j < w2; ++j) nb[(size_t)i * w2 + j] = gs[(size_t)(2 * i) * w + 2 * j];
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Laplacian and ALP (Eqs. (1)-(3))                                          */
/* ---------------------------------------------------------------------- */
/* Scale-normalised Laplacian of one Gaussian image: sigma_k^2 times the
 * 5-point stencil [0 1 0; 1 -4 1; 0 1 0], clamp-to-edge. */
void or_laplacian(const real* G, int w, int h, double sigma_k, real* L) {
    real s2 = (real)(sigma_k * sigma_k);
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            real c = G[(size_t)y * w + x];
            real up = G[(size_t)clampi(y - 1, 0, h - 1) * w + x];
            real dn = G[(size_t)clampi(y + 1, 0, h - 1) * w + x];
            real lf = G[(size_t)y * w + clampi(x - 1, 0, w - 1)];
            real rt = G[(size_t)y * w + clampi(x + 1, 0, w - 1)];
            L[(size_t)y * w + x] = s2 * (up + dn + lf + rt - (real)4 * c);
        }
}

/* Eq. (3) coefficients beta_{k,i}: the least-squares cubic through the K = S+1
 * samples (sigma_k, L_k), i.e. beta = pinv(V) with V_{k,i} = sigma_k^i.
 * Computed in double by modified Gram-Schmidt QR of V: beta = R^-1 Q^T.
 * beta is written as beta[k*4 + i]. */
int or_alp_beta(const or_params* P, double* beta) {
    int K = P->intervals + 1;
    if (K < 4 || K > 16) return -1;
    double V[16][4], Q[16][4], R[4][4];
    for (int k = 0; k < K; ++k) {
        double s = or_scale_sigma(P, k), pw = 1.0;
        for (int i = 0; i < 4; ++i) {
            V[k][i] = pw;
            pw *= s;
        }
    }
    memset(R, 0, sizeof(R));
    for (int i = 0; i < 4; ++i) {
        for (int k = 0; k < K; ++k) Q[k][i] = V[k][i];
        for (int j = 0; j < i; ++j) {
            double d = 0;
            for (int k = 0; k < K; ++k) d += Q[k][j] * Q[k][i];
            R[j][i] = d;
            for (int k = 0; k < K; ++k) Q[k][i] -= d * Q[k][j];
        }
        double nrm = 0;
        for (int k = 0; k < K; ++k) nrm += Q[k][i] * Q[k][i];
        nrm = sqrt(nrm);
        R[i][i] = nrm;
        for (int k = 0; k < K; ++k) Q[k][i] /= nrm;
    }
    /* beta^T (4 x K) = R^-1 Q^T, by back substitution per column k. */
    for (int k = 0; k < K; ++k) {
        double b[4];
        for (int i = 3; i >= 0; --i) {
            double v = Q[k][i];
            for (int j = i + 1; j < 4; ++j) v -= R[i][j] * b[j];
            b[i] = v / R[i][i];
        }
        for (int i = 0; i < 4; ++i) beta[k * 4 + i] = b[i];
    }
    return 0;
}

/* alpha_i = sum_k beta_{k,i} L_k (Eq. (3)), summed in order k = 0..K-1. */
void or_alp_fit(const real* beta_r, int K, const real* Lk, real* alpha) {
    for (int i = 0; i < 4; ++i) {
        real a = 0;
        for (int k = 0; k < K; ++k) a += beta_r[k * 4 + i] * Lk[k];
        alpha[i] = a;
    }
}

/* p(sigma) of Eq. (2), Horner form. */
static real poly(const real* a, real s) { return ((a[3] * s + a[2]) * s + a[1]) * s + a[0]; }

/* Extremal scale of the ALP cubic (Sec. III-A: solve for the zero of the
 * derivative with respect to sigma).  p'(s) = 3 a3 s^2 + 2 a2 s + a1 = 0 is
 * solved with the quadratic formula in its cancellation-free form
 * (q = -(b + sign(b) sqrt(b^2 - 4ac)) / 2; roots q/a and c/q); a = 0 leaves
 * the linear root.  A root is kept when it lies in [lo, hi) and |p| has a
 * maximum there (p * p'' < 0).  Of two kept roots the one with larger |p|
 * wins (tie: the smaller sigma).  Returns 1 and writes (sigma*, p*, p'') if
 * a root is kept, else 0. */
int or_alp_extremum(const real* a, real lo, real hi, real* s_out, real* p_out, real* pss_out) {
    real A = (real)3 * a[3], B = (real)2 * a[2], C = a[1];
    real roots[2];
    int nr = 0;
    if (A == 0) {
        if (B != 0) roots[nr++] = -C / B;
    } else {
        real disc = B * B - (real)4 * A * C;
        if (disc < 0) return 0;
        real sq = r_sqrt(disc);
        real q = (B >= 0) ? -(B + sq) / (real)2 : -(B - sq) / (real)2;
        if (q != 0) {
            roots[nr++] = q / A;
            roots[nr++] = C / q;
        } else {
            roots[nr++] = 0; /* b = 0 and disc = 0: double root at 0 */
        }
    }
    int found = 0;
    real bs = 0, bp = 0, bpss = 0;
    for (int i = 0; i < nr; ++i) {
        real s = roots[i];
        if (!(s >= lo && s < hi)) continue;
        real p = poly(a, s);
        real pss = (real)6 * a[3] * s + (real)2 * a[2];
        if (!(p * pss < 0)) continue;
        if (!found || r_abs(p) > r_abs(bp) || (r_abs(p) == r_abs(bp) && s < bs)) {
            bs = s;
            bp = p;
            bpss = pss;
            found = 1;
        }
    }
    if (found) {
        *s_out = bs;
        *p_out = bp;
        *pss_out = bpss;
    }
    return found;
}

/* Stage B of Algorithm 1: refine a candidate from the 3x3 values v[j][i]
 * (j = row -1..1, i = col -1..1, stored v[(j+1)*3 + (i+1)]) of the response
 * surface p(., ., sigma*).  One quadratic (Newton) step: offset = -H^-1 grad
 * with central differences.  Unstable candidates are dropped: det(H) <= 0,
 * tr(H)^2/det(H) >= (r+1)^2/r (edge-like), or an offset beyond max_offset on
 * either axis.  Returns 1 and writes (ox, oy, p_refined, rho) if kept. */
int or_refine3x3(const real* v, real edge_r, real max_off, real* ox, real* oy, real* pr, real* rho) {
    real c = v[4];
    real gx = (v[5] - v[3]) / (real)2;
    real gy = (v[7] - v[1]) / (real)2;
    real hxx = v[5] - (real)2 * c + v[3];
    real hyy = v[7] - (real)2 * c + v[1];
    real hxy = (v[8] - v[6] - v[2] + v[0]) / (real)4;
    real det = hxx * hyy - hxy * hxy;
    if (!(det > 0)) return 0;
    real tr = hxx + hyy;
    real ratio = tr * tr / det;
    real lim = (edge_r + (real)1) * (edge_r + (real)1) / edge_r;
    if (!(ratio < lim)) return 0;
    real dx = -(hyy * gx - hxy * gy) / det;
    real dy = -(hxx * gy - hxy * gx) / det;
    if (r_abs(dx) > max_off || r_abs(dy) > max_off) return 0;
    *ox = dx;
    *oy = dy;
    *pr = c + (gx * dx + gy * dy) / (real)2;
    *rho = ratio;
    return 1;
}

/* Stage A + B of Algorithm 1 for one octave.  For every pixel at least
 * `border` pixels from each edge: fit the cubic, find sigma*, require
 * |p*| >= T, require p* strictly above (p* > 0) or below (p* < 0) the 8
 * neighbours' cubics evaluated at the same sigma*, then refine.  Appends
 * candidates to `out` (capacity cap) and returns how many were found (which
 * may exceed cap; only the first cap are stored). */
static int detect_octave(const real* planes, int w, int h, int o, const or_params* P,
                         const real* beta_r, const uint8_t* cells, int W4, or_kp* out, int cap, int count,
                         int image) {
    int K = P->intervals + 1;
    size_t np = (size_t)w * h;
    real* L = (real*)malloc(sizeof(real) * np * K);
    real* al = (real*)malloc(sizeof(real) * np * 4);
    if (!L || !al) {
        free(L);
        free(al);
        return -1;
    }
    for (int k = 0; k < K; ++k) or_laplacian(planes + k * np, w, h, or_scale_sigma(P, k), L + k * np);
    for (size_t i = 0; i < np; ++i) {
        real lk[16], a[4];
        for (int k = 0; k < K; ++k) lk[k] = L[k * np + i];
        or_alp_fit(beta_r, K, lk, a);
        for (int j = 0; j < 4; ++j) al[i * 4 + j] = a[j];
    }
    real lo = (real)or_scale_sigma(P, 0), hi = (real)or_scale_sigma(P, P->intervals);
    real T = (real)P->contrast;
    double scale = ldexp(1.0, o);
    int b = P->border;
    for (int y = b; y <= h - 1 - b; ++y)
        for (int x = b; x <= w - 1 - b; ++x) {
            /* gated: only centres whose cell has bit o set are examined */
            if (cells && !((cells[(size_t)((y << o) >> 2) * W4 + ((x << o) >> 2)] >> o) & 1)) continue;
            real s, p, pss;
            if (!or_alp_extremum(al + ((size_t)y * w + x) * 4, lo, hi, &s, &p, &pss)) continue;
            if (!(r_abs(p) >= T)) continue;
            real v[9];
            int ext = 1;
            for (int j = -1; j <= 1 && ext; ++j)
                for (int i = -1; i <= 1; ++i) {
                    if (i == 0 && j == 0) {
                        v[4] = p;
                        continue;
                    }
                    real q = poly(al + ((size_t)(y + j) * w + (x + i)) * 4, s);
                    v[(j + 1) * 3 + (i + 1)] = q;
                    if (p > 0 ? !(q < p) : !(q > p)) {
                        ext = 0;
                        break;
                    }
                }
            if (!ext) continue;
            real ox, oy, pr, rho;
            if (!or_refine3x3(v, (real)P->edge_r, (real)P->max_offset, &ox, &oy, &pr, &rho)) continue;
            if (count < cap) {
                or_kp* k = &out[count];
                memset(k, 0, sizeof(*k));
                k->x = (double)(((real)x + ox) * (real)scale);
                k->y = (double)(((real)y + oy) * (real)scale);
                k->sigma = (double)(s * (real)scale);
                k->p = (double)pr;
                k->rho = (double)rho;
                k->pss = (double)pss;
                k->image = image;
                k->octave = o;
                k->ix = x;
                k->iy = y;
            }
            ++count;
        }
    free(L);
    free(al);
    return count;
}

/* Stages A and B over all octaves of a pyramid; returns the candidate count. */
int or_detect(const real* pyr, int W, int H, const or_params* P, int image, or_kp* out, int cap) {
    int n = or_num_octaves(W, H, P->min_side), K = P->intervals + 1;
    double beta[64];
    real beta_r[64];
    if (or_alp_beta(P, beta)) return -1;
    for (int i = 0; i < K * 4; ++i) beta_r[i] = (real)beta[i];
    int count = 0;
    for (int o = 0; o < n; ++o) {
        int w, h;
        or_octave_size(W, H, o, &w, &h);
        count = detect_octave(pyr + or_plane_offset(W, H, P, o, 0), w, h, o, P, beta_r, NULL, 0, out, cap, count,
                              image);
        if (count < 0) return count;
    }
    return count;
}

/* Stages A and B restricted by a cell mask (the learned gate, which is not
 * part of the paper).  `mask` holds one byte per 4x4-pixel cell of the base
 * image, ceil(H/4) rows of W4 = ceil(W/4) bytes.  An octave-o centre (x, y)
 * is examined only when bit o of the cell holding (x 2^o, y 2^o) / 4 is set;
 * the 3x3 comparison and the refinement still read every neighbour.  An
 * octave is examined densely (as by or_detect) when o >= 6 (bits the gate
 * never sets) or when more than fmax of the image's cells have bit o set
 * (the count against fmax x cells compared in single precision, as the
 * library does).  Returns the candidate count. */
int or_detect_masked(const real* pyr, int W, int H, const or_params* P, int image, const uint8_t* mask,
                     double fmax, or_kp* out, int cap) {
    int n = or_num_octaves(W, H, P->min_side), K = P->intervals + 1;
    int W4 = (W + 3) / 4, H4 = (H + 3) / 4;
    double beta[64];
    real beta_r[64];
    if (or_alp_beta(P, beta)) return -1;
    for (int i = 0; i < K * 4; ++i) beta_r[i] = (real)beta[i];
    int count = 0;
    for (int o = 0; o < n; ++o) {
        int w, h;
        or_octave_size(W, H, o, &w, &h);
        const uint8_t* cells = mask;
        if (o >= 6) {
            cells = NULL;
        } else {
            int64_t act = 0;
            for (int64_t c = 0; c < (int64_t)W4 * H4; ++c) act += (mask[c] >> o) & 1;
            if ((float)act > (float)fmax * (float)((int64_t)W4 * H4)) cells = NULL;
        }
        count = detect_octave(pyr + or_plane_offset(W, H, P, o, 0), w, h, o, P, beta_r, cells, W4, out, cap, count,
                              image);
        if (count < 0) return count;
    }
    return count;
}

/* Stage C of Algorithm 1: a candidate is eliminated when a candidate of an
 * adjacent octave is close to it in (x, y, sigma) and has the higher |p|.
 * Close: same sign of p, base-pixel distance at most one pixel of the coarser
 * octave (2^max(o_a, o_b)), and sigma ratio within 2^dedup_dlog2.  Ties in |p|
 * go to the finer octave.  All decisions use the pre-elimination set, so the
 * result does not depend on the order of comparison.  alive[i] = 1 if kept. */
void or_dedup(const or_kp* c, int n, const or_params* P, int32_t* alive) {
    real ratio_lim = (real)pow(2.0, P->dedup_dlog2);
    for (int i = 0; i < n; ++i) {
        alive[i] = 1;
        for (int j = 0; j < n; ++j) {
            int d = c[i].octave - c[j].octave;
            if (d != 1 && d != -1) continue;
            real pi = (real)c[i].p, pj = (real)c[j].p;
            if ((pi > 0) != (pj > 0)) continue;
            int om = c[i].octave > c[j].octave ? c[i].octave : c[j].octave;
            real lim = (real)ldexp(1.0, om);
            real dx = (real)c[i].x - (real)c[j].x, dy = (real)c[i].y - (real)c[j].y;
            if (!(dx * dx + dy * dy <= lim * lim)) continue;
            real si = (real)c[i].sigma, sj = (real)c[j].sigma;
            real shi = si > sj ? si : sj, slo = si > sj ? sj : si;
            if (!(shi <= ratio_lim * slo)) continue;
            real ai = r_abs(pi), aj = r_abs(pj);
            if (aj > ai || (aj == ai && c[j].octave < c[i].octave)) {
                alive[i] = 0;
                break;
            }
        }
    }
}

/* Canonical order: |p| descending, then octave, iy, ix ascending. */
static int cmp_canonical(const void* pa, const void* pb) {
    const or_kp* a = (const or_kp*)pa;
    const or_kp* b = (const or_kp*)pb;
    real aa = r_abs((real)a->p), ab = r_abs((real)b->p);
    if (aa != ab) return aa > ab ? -1 : 1;
    if (a->octave != b->octave) return a->octave < b->octave ? -1 : 1;
    if (a->iy != b->iy) return a->iy < b->iy ? -1 : 1;
    if (a->ix != b->ix) return a->ix < b->ix ? -1 : 1;
    return 0;
}

/* Keep the alive candidates, sort canonically, keep the first topk (all if
 * topk <= 0).  Returns the number written to out. */
int or_select(const or_kp* c, int n, const int32_t* alive, int topk, or_kp* out) {
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (alive[i]) out[m++] = c[i];
    qsort(out, (size_t)m, sizeof(or_kp), cmp_canonical);
    if (topk > 0 && m > topk) m = topk;
    return m;
}

/* Gradient of a Gaussian image at an interior pixel (central differences,
 * y pointing down), its magnitude and angle in [0, 2 pi). */
static void grad(const real* G, int w, int u, int v, real* mag, real* ang) {
    real gx = G[(size_t)v * w + u + 1] - G[(size_t)v * w + u - 1];
    real gy = G[(size_t)(v + 1) * w + u] - G[(size_t)(v - 1) * w + u];
    *mag = r_sqrt(gx * gx + gy * gy);
    real a = r_atan2(gy, gx);
    if (a < 0) a += (real)TWO_PI;
    if (a >= (real)TWO_PI) a -= (real)TWO_PI;
    *ang = a;
}

/* Index of the scale image a keypoint of octave-relative scale s reads:
 * the nearest k, clamp(round(S * log2(s / sigma0)), 0, S). */
int or_scale_index(const or_params* P, double s_oct) {
    real t = (real)P->intervals * r_log2((real)s_oct / (real)P->sigma0);
    int k = (int)r_floor(t + (real)0.5);
    return clampi(k, 0, P->intervals);
}

/* Algorithm 2 stage A for one keypoint: the 36-bin histogram of gradient
 * angles over the integer pixels strictly inside radius ori_radius*sigma of
 * the (sub-pixel) keypoint, each weighted by its gradient magnitude and a
 * Gaussian of sigma ori_wsigma*sigma, split linearly between the two nearest
 * bins (bin b is centred on angle b * 2 pi / 36).  Pixels need all four
 * gradient neighbours inside the image.  hist has ori_bins entries. */
void or_orient_hist(const real* G, int w, int h, double cx_d, double cy_d, double s_d,
                    const or_params* P, real* hist) {
    int nb = P->ori_bins;
    real cx = (real)cx_d, cy = (real)cy_d, s = (real)s_d;
    for (int b = 0; b < nb; ++b) hist[b] = 0;
    real R = (real)P->ori_radius * s;
    real R2 = R * R;
    real ws = (real)P->ori_wsigma * s;
    real den = (real)2 * ws * ws;
    int u0 = (int)ceil((double)(cx - R)), u1 = (int)floor((double)(cx + R));
    int v0 = (int)ceil((double)(cy - R)), v1 = (int)floor((double)(cy + R));
    if (u0 < 1) u0 = 1;
    if (v0 < 1) v0 = 1;
    if (u1 > w - 2) u1 = w - 2;
    if (v1 > h - 2) v1 = h - 2;
    for (int v = v0; v <= v1; ++v)
        for (int u = u0; u <= u1; ++u) {
            real dx = (real)u - cx, dy = (real)v - cy;
            real d2 = dx * dx + dy * dy;
            if (!(d2 < R2)) continue;
            real mag, ang;
            grad(G, w, u, v, &mag, &ang);
            real wt = mag * r_exp(-d2 / den);
            real fb = ang * (real)nb / (real)TWO_PI;
            real f0 = r_floor(fb);
            real fr = fb - f0;
            int b0 = ((int)f0 % nb + nb) % nb;
            int b1 = (b0 + 1) % nb;
            hist[b0] += wt * ((real)1 - fr);
            hist[b1] += wt * fr;
        }
}

/* Dominant orientations from a histogram: bins that are strict circular local
 * maxima with value > ori_peak * max, highest first (tie: lower bin), at most
 * max_ori; each refined by a parabola through the bin and its neighbours.
 * Writes angles in [0, 2 pi) and peak heights; returns the count. */
int or_orient_peaks(const real* hist, const or_params* P, real* theta, real* peak) {
    int nb = P->ori_bins, cnt = 0;
    real mx = 0;
    for (int b = 0; b < nb; ++b)
        if (hist[b] > mx) mx = hist[b];
    real thr = (real)P->ori_peak * mx;
    int idx[64];
    for (int b = 0; b < nb; ++b) {
        real c = hist[b], l = hist[(b + nb - 1) % nb], r = hist[(b + 1) % nb];
        if (c > l && c > r && c > thr) idx[cnt++] = b;
    }
    /* order by height, descending; stable on bin index */
    for (int i = 1; i < cnt; ++i) {
        int t = idx[i], j = i - 1;
        while (j >= 0 && hist[idx[j]] < hist[t]) {
            idx[j + 1] = idx[j];
            --j;
        }
        idx[j + 1] = t;
    }
    if (cnt > P->max_ori) cnt = P->max_ori;
    for (int i = 0; i < cnt; ++i) {
        int b = idx[i];
        real c = hist[b], l = hist[(b + nb - 1) % nb], r = hist[(b + 1) % nb];
        real off = (real)0.5 * (l - r) / (l - (real)2 * c + r);
        real t = ((real)b + off) * (real)TWO_PI / (real)nb;
        if (t < 0) t += (real)TWO_PI;
        if (t >= (real)TWO_PI) t -= (real)TWO_PI;
        theta[i] = t;
        peak[i] = c;
    }
    return cnt;
}

/* Orientation assignment for a canonical keypoint list: each keypoint becomes
 * one record per dominant orientation (in peak order); the expanded list stays
 * in input order and is cut at topk (all if <= 0).  Keypoints whose histogram
 * has no peak are dropped.  Returns the number of records written. */
int or_orient(const real* pyr, int W, int H, const or_params* P, const or_kp* kp, int n, or_kp* out,
              int cap) {
    int m = 0;
    real hist[64], th[64], pk[64];
    for (int i = 0; i < n; ++i) {
        int o = kp[i].octave, w, h;
        or_octave_size(W, H, o, &w, &h);
        double sc = ldexp(1.0, -o);
        double cx = (double)((real)kp[i].x * (real)sc), cy = (double)((real)kp[i].y * (real)sc);
        double s = (double)((real)kp[i].sigma * (real)sc);
        int k = or_scale_index(P, s);
        or_orient_hist(pyr + or_plane_offset(W, H, P, o, k), w, h, cx, cy, s, P, hist);
        int c = or_orient_peaks(hist, P, th, pk);
        for (int j = 0; j < c; ++j) {
            if (P->topk > 0 && m >= P->topk) return m;
            if (m >= cap) return m;
            out[m] = kp[i];
            out[m].theta = (double)th[j];
            out[m].peak = (double)pk[j];
            ++m;
        }
    }
    return m;
}

/* Algorithm 2 stage B for one oriented keypoint: the 4x4-cell x 8-bin
 * histogram.  Pixel offsets from the keypoint are rotated by -theta and
 * measured in cells of desc_cell*sigma; gradient angles are taken relative
 * to theta.  Integer pixels strictly inside desc_radius*sigma contribute
 * magnitude x Gaussian(desc_wsigma*sigma) split trilinearly between the two
 * nearest cells in each direction (cell centres at -1.5, -0.5, 0.5, 1.5) and
 * the two nearest of 8 orientation bins (bin b centred on b * 2 pi / 8).
 * Index = (row*4 + col)*8 + bin.  Then L2-normalise, clamp at desc_clamp,
 * L2-normalise again; an all-zero histogram stays zero. */
void or_descriptor(const real* G, int w, int h, double cx_d, double cy_d, double s_d, double th_d,
                   const or_params* P, real* d) {
    real cx = (real)cx_d, cy = (real)cy_d, s = (real)s_d, th = (real)th_d;
    for (int i = 0; i < 128; ++i) d[i] = 0;
    real ct = IS_F32 ? (real)cosf((float)th) : (real)cos((double)th);
    real st = IS_F32 ? (real)sinf((float)th) : (real)sin((double)th);
    real R = (real)P->desc_radius * s;
    real R2 = R * R;
    real cw = (real)P->desc_cell * s;
    real ws = (real)P->desc_wsigma * s;
    real den = (real)2 * ws * ws;
    int u0 = (int)ceil((double)(cx - R)), u1 = (int)floor((double)(cx + R));
    int v0 = (int)ceil((double)(cy - R)), v1 = (int)floor((double)(cy + R));
    if (u0 < 1) u0 = 1;
    if (v0 < 1) v0 = 1;
    if (u1 > w - 2) u1 = w - 2;
    if (v1 > h - 2) v1 = h - 2;
    for (int v = v0; v <= v1; ++v)
        for (int u = u0; u <= u1; ++u) {
            real dx = (real)u - cx, dy = (real)v - cy;
            real d2 = dx * dx + dy * dy;
            if (!(d2 < R2)) continue;
            real rx = (ct * dx + st * dy) / cw;
            real ry = (ct * dy - st * dx) / cw;
            real mag, ang;
            grad(G, w, u, v, &mag, &ang);
            real rel = ang - th;
            if (rel < 0) rel += (real)TWO_PI;
            if (rel >= (real)TWO_PI) rel -= (real)TWO_PI;
            real wt = mag * r_exp(-d2 / den);
            real fx = rx + (real)1.5, fy = ry + (real)1.5, fo = rel * (real)8 / (real)TWO_PI;
            real x0f = r_floor(fx), y0f = r_floor(fy), o0f = r_floor(fo);
            real ax = fx - x0f, ay = fy - y0f, ao = fo - o0f;
            int x0 = (int)x0f, y0 = (int)y0f, o0 = (int)o0f;
            for (int jy = 0; jy < 2; ++jy) {
                int yy = y0 + jy;
                if (yy < 0 || yy > 3) continue;
                real wy = jy ? ay : (real)1 - ay;
                for (int jx = 0; jx < 2; ++jx) {
                    int xx = x0 + jx;
                    if (xx < 0 || xx > 3) continue;
                    real wx = jx ? ax : (real)1 - ax;
                    for (int jo = 0; jo < 2; ++jo) {
                        int oo = ((o0 + jo) % 8 + 8) % 8;
                        real wo = jo ? ao : (real)1 - ao;
                        d[(yy * 4 + xx) * 8 + oo] += wt * wy * wx * wo;
                    }
                }
            }
        }
    real n2 = 0;
    for (int i = 0; i < 128; ++i) n2 += d[i] * d[i];
    if (!(n2 > 0)) return;
    real inv = (real)1 / r_sqrt(n2);
    real cl = (real)P->desc_clamp;
    for (int i = 0; i < 128; ++i) {
        real t = d[i] * inv;
        d[i] = t > cl ? cl : t;
    }
    n2 = 0;
    for (int i = 0; i < 128; ++i) n2 += d[i] * d[i];
    inv = (real)1 / r_sqrt(n2);
    for (int i = 0; i < 128; ++i) d[i] = d[i] * inv;
}

/* Descriptors for a list of oriented keypoints; desc is n x 128 doubles. */
void or_describe(const real* pyr, int W, int H, const or_params* P, const or_kp* kp, int n, double* desc) {
    real d[128];
    for (int i = 0; i < n; ++i) {
        int o = kp[i].octave, w, h;
        or_octave_size(W, H, o, &w, &h);
        double sc = ldexp(1.0, -o);
        double cx = (double)((real)kp[i].x * (real)sc), cy = (double)((real)kp[i].y * (real)sc);
        double s = (double)((real)kp[i].sigma * (real)sc);
        int k = or_scale_index(P, s);
        or_descriptor(pyr + or_plane_offset(W, H, P, o, k), w, h, cx, cy, s, kp[i].theta, P, d);
        for (int j = 0; j < 128; ++j) desc[(size_t)i * 128 + j] = (double)d[j];
    }
}

/* The whole front half for one image: pyramid, detection (stages A-B),
 * deduplication (stage C), top-k, orientation, descriptors.
 * out_kp / out_desc have room for `cap` records; stats (may be NULL) gets
 * {candidates, after dedup, after top-k, oriented}.  Returns the number of
 * oriented keypoints written, or a negative value on failure. */
int or_run(const uint8_t* img, int W, int H, int pitch, const or_params* P, int image, or_kp* out_kp,
           double* out_desc, int cap, int32_t* stats) {
    int64_t len = or_pyramid_len(W, H, P);
    real* pyr = (real*)malloc(sizeof(real) * (size_t)len);
    if (!pyr) return -1;
    if (or_pyramid(img, W, H, pitch, P, pyr)) {
        free(pyr);
        return -1;
    }
    int ccap = 1 << 16;
    or_kp* cand = (or_kp*)malloc(sizeof(or_kp) * ccap);
    int32_t* alive = (int32_t*)malloc(sizeof(int32_t) * ccap);
    or_kp* sel = (or_kp*)malloc(sizeof(or_kp) * ccap);
    if (!cand || !alive || !sel) {
        free(pyr);
        free(cand);
        free(alive);
        free(sel);
        return -1;
    }
    int nc = or_detect(pyr, W, H, P, image, cand, ccap);
    if (nc > ccap) nc = ccap;
    or_dedup(cand, nc, P, alive);
    int na = 0;
    for (int i = 0; i < nc; ++i) na += alive[i];
    int ns = or_select(cand, nc, alive, P->topk, sel);
    int no = or_orient(pyr, W, H, P, sel, ns, out_kp, cap);
    if (out_desc) or_describe(pyr, W, H, P, out_kp, no, out_desc);
    if (stats) {
        stats[0] = nc;
        stats[1] = na;
        stats[2] = ns;
        stats[3] = no;
    }
    free(pyr);
    free(cand);
    free(alive);
    free(sel);
    return no;
}
