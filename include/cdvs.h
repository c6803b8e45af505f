/*
 * cdvs.h -- C ABI of the MI355X (gfx950) CDVS front half.
 *
 * The front half of a CDVS encoder ("Fast MPEG-CDVS Encoder with GPU-CPU
 * Hybrid Computing", Duan et al.): Gaussian scale space, ALP keypoint
 * detection, orientation assignment and the 128-D local descriptor, over a
 * batch of 8-bit grayscale images.  Selection by relevance, compression and
 * aggregation stay with the caller.
 *
 * Conventions for every call below
 *   - Pointers prefixed d_ are device pointers (HIP device memory of the
 *     current device); all others are host pointers.
 *   - Device buffers passed in are owned by the caller; the library never
 *     frees or retains them past the call.  The context owns only its own
 *     small tables and scratch, allocated once by cdvs_ctx_create.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Compute calls only
 *     enqueue work on it and return; they never synchronise, never allocate,
 *     and may be captured into a HIP graph.  Errors detectable on the host
 *     (null pointers, bad sizes, bad parameters) are returned at once and
 *     nothing is enqueued.  Conditions only the device can see (a capacity
 *     overflow) are latched in the context and returned by cdvs_sync_status.
 *   - Two calls on the same context must not run concurrently (they share
 *     the context's scratch); use one context per stream.
 *   - Coordinates: pixel centres are at integers, x to the right, y down.
 *     A keypoint of octave o has base-image coordinates (ix + dx) * 2^o.
 */
#ifndef CDVS_H
#define CDVS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CDVS_OK = 0,
    CDVS_ERR_ARG = -1,      /* null pointer, unsupported parameter value */
    CDVS_ERR_SHAPE = -2,    /* image size, pitch or count out of range */
    CDVS_ERR_CAPACITY = -3, /* results were truncated; what was written is valid */
    CDVS_ERR_HIP = -4,      /* a HIP runtime call failed (message in cdvs_last_error) */
    CDVS_ERR_STATE = -5,    /* call out of order (e.g. no context) */
    CDVS_ERR_VERSION = -6   /* params.version does not match CDVS_PARAMS_VERSION */
} cdvs_status;

#define CDVS_PARAMS_VERSION 2
#define CDVS_DESC_DIM 128
#define CDVS_MIN_SIDE 16
#define CDVS_MAX_SIDE 8192
#define CDVS_MAX_IMAGES 65536
#define CDVS_MAX_KP_CAPACITY 8192 /* per image */

/* Method constants.  sigma0 and intervals are fixed by the compiled
 * kernels (1.6 and 4: five scale images per octave, Gaussian radii 7, 5, 7,
 * 9, 12); the others are read at run time.  Defaults: cdvs_default_params. */
typedef struct {
    int32_t version;     /* CDVS_PARAMS_VERSION */
    float sigma0;        /* base scale of each octave (octave pixels): 1.6 */
    int32_t intervals;   /* scale intervals per octave: 4 (images k = 0..4) */
    int32_t min_side;    /* octaves continue until one has a short side < this: 32 */
    float contrast;      /* minimum |p| of a candidate, 0..255 intensity scale: 1.5 */
    float edge_r;        /* reject when tr(H)^2/det(H) >= (r+1)^2/r: 10 */
    int32_t border;      /* detection margin in octave pixels: 4 */
    float max_offset;    /* reject a refinement offset beyond this per axis: 0.5 */
    float dedup_dlog2;   /* cross-octave duplicates: |log2 sigma ratio| <= this: 0.25 */
    float ori_radius;    /* orientation window radius / sigma: 3.96 */
    float ori_wsigma;    /* orientation Gaussian weight sigma / sigma: 1.5 */
    float ori_peak;      /* keep peaks above this fraction of the highest: 0.8 */
    int32_t max_ori;     /* orientations per keypoint, 1..4: 4 */
    float desc_cell;     /* descriptor cell side / sigma: 3 */
    float desc_radius;   /* descriptor window radius / sigma: 6 */
    float desc_wsigma;   /* descriptor Gaussian weight sigma / sigma: 6 */
    float desc_clamp;    /* clamp after the first L2 normalisation: 0.2 */
    int32_t topk;        /* keypoints kept per image (<= kp capacity): 1000 */
    float mask_fmax;     /* gated detection: an (image, octave) whose mask has more
                            than this fraction of active cells is examined densely: 0.6 */
} cdvs_params;

/* One u8 image inside the caller's packed image buffer: byte offset of its
 * first row, width and height in pixels, row pitch in bytes (>= width). */
typedef struct {
    int64_t offset;
    int32_t width, height, pitch;
    int32_t reserved; /* 0 */
} cdvs_image_desc;

/* 48-byte keypoint record (relevance features of Sec. III-B, Eq. (5):
 * sigma, p, rho, p_ss; distance to the image centre follows from x, y). */
typedef struct {
    float x, y;      /* base-image pixels */
    float sigma;     /* scale in base-image pixels */
    float p;         /* ALP response at (x, y, sigma), refined */
    float theta;     /* orientation in [0, 2 pi) (0 before cdvs_orient) */
    float rho;       /* tr(H)^2 / det(H) of the response surface */
    float p_ss;      /* d^2 p / d sigma^2 at the extremum (octave units) */
    float peak;      /* orientation histogram peak height (0 before cdvs_orient) */
    int32_t image;   /* index of the image in the batch */
    int32_t octave;  /* octave o */
    int32_t ix, iy;  /* integer position of the candidate in octave pixels */
} cdvs_keypoint;

typedef struct cdvs_ctx cdvs_ctx;

/* Defaults listed in cdvs_params. */
cdvs_params cdvs_default_params(void);

/* Host-only check of a batch description and parameters; touches no device.
 * Returns CDVS_OK or the error cdvs_ctx_create would return.  `msg` (may be
 * NULL) receives a NUL-terminated reason, at most msg_len bytes. */
cdvs_status cdvs_validate(const cdvs_params* params, const cdvs_image_desc* images, int32_t n_images,
                          int32_t kp_capacity, char* msg, int32_t msg_len);

/* Create a context for one batch layout: n_images images described by the
 * host array `images` (copied).  kp_capacity is the per-image record count
 * of every keypoint buffer passed to the calls below (topk <= kp_capacity).
 * Allocates the context's device tables and scratch on the current device
 * (scratch is about 0.4 MB per image).  On failure *out is NULL. */
cdvs_status cdvs_ctx_create(const cdvs_params* params, const cdvs_image_desc* images, int32_t n_images,
                            int32_t kp_capacity, cdvs_ctx** out);
void cdvs_ctx_destroy(cdvs_ctx* ctx);

/* Reason for the last error of a context (or of the last failed
 * cdvs_ctx_create when ctx is NULL).  Valid until the next call. */
const char* cdvs_last_error(const cdvs_ctx* ctx);

/* Size in bytes of the pyramid buffer (all images, octaves and scales). */
int64_t cdvs_pyramid_bytes(const cdvs_ctx* ctx);
int32_t cdvs_num_octaves(const cdvs_ctx* ctx, int32_t image);

/* Where plane G_{o,k} of image `image` lives in the pyramid buffer: offset
 * in floats from its start, width, height and row pitch in floats. */
cdvs_status cdvs_plane_layout(const cdvs_ctx* ctx, int32_t image, int32_t octave, int32_t k,
                              int64_t* offset, int32_t* width, int32_t* height, int32_t* pitch);

/* Scale space (Sec. III-A, Eq. (1); Sec. IV-A, Algorithm 1 stage A and its
 * downsampling step).  Reads the packed u8 images at d_images (layout given
 * at context creation) and writes every G_{o,k}, k = 0..4, as FP32 planes
 * on the 0..255 scale into d_pyr (cdvs_pyramid_bytes bytes, 256-byte
 * aligned).  G_{0,0} is the input blurred by sigma0 (the input is taken as
 * sharp); G_{o,k} is G_{o,0} blurred by sigma0 sqrt(2^(k/2) - 1); G_{o+1,0}
 * takes the even samples of G_{o,4}.  Separable, vertical pass first,
 * clamp-to-edge borders. */
cdvs_status cdvs_pyramid(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, void* stream);

/* ALP detection (Sec. III-A, Eqs. (2)-(3); Algorithm 1 stages A-C) on a
 * pyramid written by cdvs_pyramid.  Per pixel: scale-normalised 5-point
 * Laplacians L_k, the least-squares cubic p(sigma) through them, its extremal
 * scale in [sigma_0, sigma_4) where |p| peaks, |p| >= contrast, a strict
 * extremum against the 8 neighbours' cubics at the same scale, then one
 * quadratic refinement step (unstable candidates dropped).  Candidates of
 * adjacent octaves that are close in (x, y, sigma) with the same sign keep
 * only the higher |p|.  Writes per image the topk strongest keypoints in
 * canonical order (|p| desc, octave, iy, ix asc) to d_kp[image][0..] and
 * their number to d_count[image].  d_kp: n_images x kp_capacity records,
 * d_count: n_images int32.
 * d_mask (NULL = every pixel): one byte per 4x4 cell of each base image (the
 * cell layout of cdvs_cnn_cell_layout); an octave-o pixel (x, y) is examined
 * only when bit o of the cell holding (x 2^o, y 2^o) / 4 is set -- neighbours
 * are still read in full -- unless more than mask_fmax of that image's cells
 * have bit o set, in which case octave o of that image is examined densely.
 * Octaves 6 and up (images whose short side exceeds 992 px have them) have
 * no mask bit and are always examined densely.
 * Each image holds up to max(8192, W*H/64 rounded up to 256) candidates
 * before stage C; one that finds more than its capacity keeps those stored
 * and latches an overflow.  Stage C and the top-k work on at most 8192
 * candidates per image: an image with more is first cut to its 8192 largest
 * |p|, which leaves the result unchanged whenever its last kept keypoint is
 * stronger than the weakest of those (a candidate is only ever removed by a
 * stronger one); when it is not, the image is latched as inexact.
 * d_pyr must be 256-byte aligned (as cdvs_pyramid requires), else
 * CDVS_ERR_ARG. */
cdvs_status cdvs_alp_detect(cdvs_ctx* ctx, const float* d_pyr, const uint8_t* d_mask, cdvs_keypoint* d_kp,
                            int32_t* d_count, void* stream);

/* Orientation assignment (Sec. III-B and IV-B, Algorithm 2 stage A): for
 * each input keypoint a 36-bin histogram of gradient angles of G_{o,k*}
 * (k* the nearest scale image) over pixels strictly within ori_radius*sigma,
 * weighted by magnitude and a Gaussian of ori_wsigma*sigma, split linearly
 * between neighbouring bins; every strict local maximum above ori_peak x the
 * highest gives one output record (at most max_ori, highest first), its angle
 * refined by a parabola.  Output per image: records in input order, cut at
 * topk.  d_kp_in/d_count_in as written by cdvs_alp_detect; d_kp_out and
 * d_count_out have the same shapes and must not alias the inputs.  An input
 * record whose octave is outside 0..15, whose x or y is not finite, or whose
 * scale in octave units, sigma / 2^octave, is not in (0, 2 sigma0] (detected
 * keypoints have sigma0 <= that < 2 sigma0) gets no orientation. */
cdvs_status cdvs_orient(cdvs_ctx* ctx, const float* d_pyr, const cdvs_keypoint* d_kp_in,
                        const int32_t* d_count_in, cdvs_keypoint* d_kp_out, int32_t* d_count_out,
                        void* stream);

/* Local descriptor (Sec. III-B and IV-B, Algorithm 2 stage B): for each
 * oriented keypoint, the 4x4-cell x 8-bin histogram of gradient angles
 * relative to theta over pixels strictly within desc_radius*sigma, offsets
 * rotated by -theta and measured in cells of desc_cell*sigma, weighted by
 * magnitude and a Gaussian of desc_wsigma*sigma, split trilinearly; then
 * L2-normalised, clamped at desc_clamp and L2-normalised again.  Element
 * (row*4 + col)*8 + bin.  d_desc: n_images x kp_capacity x 128 floats; rows
 * at or beyond d_count[image] are left untouched.  A record that
 * cdvs_orient would not take (see there) gets an all-zero descriptor. */
cdvs_status cdvs_describe(cdvs_ctx* ctx, const float* d_pyr, const cdvs_keypoint* d_kp, const int32_t* d_count,
                          float* d_desc, void* stream);

/* Synchronise `stream`, then return CDVS_ERR_SHAPE if any call since the
 * last cdvs_sync_status latched a front-end source that does not fit (see
 * cdvs_front_end), else CDVS_ERR_CAPACITY if one latched a candidate
 * overflow or an inexact top-k (see cdvs_alp_detect), else CDVS_OK; clears
 * the latch.  The only blocking call. */
cdvs_status cdvs_sync_status(cdvs_ctx* ctx, void* stream);

/* Smallest candidate capacity over the context's images (pre-deduplication
 * candidates: max(8192, W*H/64 rounded up to 256) per image). */
int32_t cdvs_candidate_capacity(const cdvs_ctx* ctx);

/* HIP graph of one whole pass.  cdvs_graph_capture records cdvs_pyramid,
 * cdvs_alp_detect (plain), cdvs_orient and cdvs_describe on the given
 * buffers into a graph owned by the context (capturing on a stream of its
 * own; nothing runs), replacing any previous one.  cdvs_graph_launch enqueues
 * one replay on `stream`; the buffers must stay valid while the graph exists.
 * Capture is refused while event timing is enabled (CDVS_ERR_STATE) and for
 * a null pointer (CDVS_ERR_ARG), keeping any previous graph; an argument
 * that one of the recorded calls refuses (a misaligned pyramid) ends the
 * capture with that call's error, and the context then holds no graph.
 * The graph holds only kernel nodes (counters are cleared by a kernel,
 * never by a memset). */
cdvs_status cdvs_graph_capture(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, cdvs_keypoint* d_kp,
                               int32_t* d_count, cdvs_keypoint* d_kp_ori, int32_t* d_count_ori, float* d_desc);
/* The same for the gated pass (detection gated by the learned candidate mask):
 * cdvs_cnn_forward with the fused inference kernel (d_mask: the caller's
 * buffer of cdvs_cnn_cells bytes, bits at threshold tau in (0, 1); d_params:
 * CDVS_CNN_PARAMS fp32), then the four calls above with d_mask passed to
 * cdvs_alp_detect.  A tau outside (0, 1) is refused like a null pointer,
 * before the capture begins; otherwise the errors are as above. */
cdvs_status cdvs_graph_capture_gated(cdvs_ctx* ctx, const uint8_t* d_images, const float* d_params, float tau,
                                     uint8_t* d_mask, float* d_pyr, cdvs_keypoint* d_kp, int32_t* d_count,
                                     cdvs_keypoint* d_kp_ori, int32_t* d_count_ori, float* d_desc);
cdvs_status cdvs_graph_launch(cdvs_ctx* ctx, void* stream);

/* Autotuning of two kernels on the context's batch.  CDVS_KERNEL_SCALES has
 * CDVS_TUNE_VARIANTS tile shapes (64x32, 128x16, 32x32, 64x16; every shape
 * produces bit-identical planes); CDVS_KERNEL_DETECT has
 * CDVS_DETECT_VARIANTS launch forms (0: one wave per strip, dispatched by the
 * hardware; 1: persistent, a fixed grid pulling strips from per-XCD work
 * counters; both find the same candidates).  cdvs_autotune times each
 * shape with cdvs_pyramid on the given buffers, then each launch form of the
 * ungated detection on the resulting pyramid (candidates go to the
 * context's scratch; d_pyr must be 256-byte aligned), 2 warm-ups + 7
 * timed runs each, the variants taken in turn, median; blocking; it keeps
 * the fastest of each.  With
 * cache_path (may be NULL) a JSON file keyed by (GPU arch, image size,
 * batch-size bucket) is read first (a hit skips the timing) and updated
 * after timing.  cdvs_tune_get / cdvs_tune_set read and force a kernel's
 * variant.  A captured graph keeps the variants selected when it was
 * captured.  The cache file is a JSON object with one "key": {...} entry per
 * line; an unreadable file is treated as empty and rewritten. */
#define CDVS_TUNE_VARIANTS 4
#define CDVS_DETECT_VARIANTS 2
cdvs_status cdvs_autotune(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, const char* cache_path,
                          void* stream);
int32_t cdvs_tune_get(const cdvs_ctx* ctx, int32_t kernel);
cdvs_status cdvs_tune_set(cdvs_ctx* ctx, int32_t kernel, int32_t variant);

/* ---------------------------------------------------------------------- */
/* BMLoG scale space (Sec. III-A): the comparison variant of cdvs_pyramid   */
/* ---------------------------------------------------------------------- */
/* Writes the same planes as cdvs_pyramid, into the same layout, by the
 * block-based mixture-domain filtering the paper compares: each octave image
 * is cut into 128 x 128 blocks overlapping by 16 pixels on every side
 * (block (bx, by) covers columns 96 bx - 16 .. 96 bx + 111 and rows likewise,
 * pixels outside the image taken from the nearest edge pixel; a 640x480
 * image has 35); every block is transformed once (2-D DFT), multiplied by
 * the separable transfer function of each Gaussian (the DFT of its
 * normalised taps, radius ceil(4 s), placed on the 128-periodic grid) and
 * transformed back once per scale image, keeping its central 96 x 96
 * pixels.  Octave 0 filters the u8 input with g0 (G_{0,0}) and with g0
 * then g_k (G_{0,k}): one forward and five inverse transforms per block;
 * octave o >= 1 filters G_{o,0} (G_{o-1,4} at even pixels) with g_1..g_4.
 * The Laplacian stays in the spatial domain: cdvs_alp_detect runs on the
 * result unchanged.  Where a kernel's radius is at most 16 (all but the
 * octave-0 combined kernels, radius up to 19, whose wrapped tail is below
 * 1e-6 of their mass) the kept pixels equal the spatial filter up to
 * rounding; near the image border octave 0 differs from cdvs_pyramid's
 * two clamped passes by the one clamped combined pass.  FP32 transforms:
 * planes within about 1e-3 of the exact block result on the 0..255 scale.
 * d_pyr: 256-byte aligned, cdvs_pyramid_bytes long.  One launch per octave;
 * uses 134 KB of LDS per workgroup. */
cdvs_status cdvs_pyramid_bmlog(cdvs_ctx* ctx, const uint8_t* d_images, float* d_pyr, void* stream);

/* ---------------------------------------------------------------------- */
/* Front end (Sec. III: inputs reduced to a longer side of at most 640)     */
/* ---------------------------------------------------------------------- */
#define CDVS_FRONT_LONG_SIDE 640

/* Output size of the front end for a width x height input (1..CDVS_MAX_SIDE
 * per side, else CDVS_ERR_SHAPE): unchanged when the longer side L is at
 * most 640; otherwise the longer side becomes 640 and the shorter one
 * round(S * 640 / L) (half up), at least 1.  A context for front-end output
 * is created with these sizes. */
cdvs_status cdvs_front_size(int32_t width, int32_t height, int32_t* out_width, int32_t* out_height);

/* Brings source image i (d_src_desc[i], a device array of the context's
 * image count; offsets into d_src) down to the context's image i, written
 * into d_images at that image's offset and pitch.  Area averaging: every
 * output pixel is the mean of the source over its footprint, each source
 * pixel weighted by its overlap area, computed in exact integers and
 * rounded half up (along an axis of n source and m output pixels, source
 * pixel i spans [i m, (i+1) m) and output pixel j spans [j n, (j+1) n);
 * output = floor((2 N + W H) / (2 W H)) for the integer weighted sum N).
 * An image whose longer side is at most 640 is copied.  A source whose size
 * (by cdvs_front_size) is not the context's image size, or whose
 * descriptor is invalid, is skipped and latched: cdvs_sync_status returns
 * CDVS_ERR_SHAPE.  d_images must not alias d_src.  The source table is
 * read on the device: the caller guarantees that every source it describes
 * lies inside d_src (the library does not know that buffer's size). */
cdvs_status cdvs_front_end(cdvs_ctx* ctx, const uint8_t* d_src, const cdvs_image_desc* d_src_desc,
                           uint8_t* d_images, void* stream);

/* ---------------------------------------------------------------------- */
/* Keypoint selection by relevance (Sec. III-B, Eqs. (4)-(5))               */
/* ---------------------------------------------------------------------- */
#define CDVS_REL_FEATURES 5
#define CDVS_REL_EDGES 15
#define CDVS_REL_BINS 16

/* The relevance tables, device buffers (float32) owned by the caller: for
 * characteristic c = 0..4 (sigma in base pixels, |p|, distance to the image
 * centre, rho, p_ss -- in that order), d_edges[c][0..14] increasing bin
 * edges and d_values[c][0..15] table values (positive). */
typedef struct {
    const float* d_edges;
    const float* d_values;
} cdvs_relevance_model;

/* Keeps, per image, the n_keep keypoints of highest relevance
 *   r = f_0(sigma) f_1(|p|) f_2(d) f_3(rho) f_4(p_ss),
 * f_c(v) = d_values[c][b], b = the number of d_edges[c] entries <= v,
 * d = distance of (x, y) from ((W-1)/2, (H-1)/2) over that point's distance
 * to a corner, all in single precision (the product left to right).  Input:
 * the first d_count_in[image] records of d_kp_in[image] (clamped to
 * 0..kp_capacity; e.g. cdvs_alp_detect's output with a large topk).
 * Output: the kept records in order of r, descending (equal r: input
 * order), in d_kp_out[image][0..], their number min(count, n_keep) in
 * d_count_out[image], and (d_score may be NULL) their r in
 * d_score[image][0..] (n_images x kp_capacity floats).  Outputs must not
 * alias inputs; 1 <= n_keep. */
cdvs_status cdvs_relevance_select(cdvs_ctx* ctx, const cdvs_relevance_model* model, const cdvs_keypoint* d_kp_in,
                                  const int32_t* d_count_in, int32_t n_keep, cdvs_keypoint* d_kp_out,
                                  int32_t* d_count_out, float* d_score, void* stream);

/* ---------------------------------------------------------------------- */
/* Descriptor compression: transform coding and ternary quantisation        */
/* (Sec. III-C)                                                              */
/* ---------------------------------------------------------------------- */
#define CDVS_TQ_WORDS 8   /* 32-bit code words per descriptor (up to 128 elements x 2 bits) */

/* The quantiser, device buffers owned by the caller: per transformed
 * element e (0..127), thresholds d_lo[e] <= d_hi[e] (float32), and a
 * priority order d_order[0..127] (int32, a permutation of 0..127). */
typedef struct {
    const float* d_lo;
    const float* d_hi;
    const int32_t* d_order;
} cdvs_tq_model;

/* Codes the first d_count[image] descriptors of every image (d_desc as
 * cdvs_describe writes it, 16-byte aligned).  Cell c = 4 row + col of a
 * descriptor (bins h_0..h_7 at elements 8c..8c+7) is transformed by set A
 * when row + col is even and by set B otherwise:
 *   A: v0 = (h2-h6)/2, v1 = (h3-h7)/2, v2 = (h0-h1)/2, v3 = (h2-h3)/2,
 *      v4 = (h4-h5)/2, v5 = (h6-h7)/2, v6 = ((h0+h4)-(h2+h6))/4,
 *      v7 = ((h0+h2+h4+h6)-(h1+h3+h5+h7))/8;
 *   B: v0 = (h0-h4)/2, v1 = (h1-h5)/2, v2 = (h7-h0)/2, v3 = (h1-h2)/2,
 *      v4 = (h3-h4)/2, v5 = (h5-h6)/2, v6 = ((h1+h5)-(h3+h7))/4,
 *      v7 = ((h0+h1+h2+h3)-(h4+h5+h6+h7))/8
 * (each evaluated left to right in single precision), element 8c + k being
 * v_k; element e becomes +1 if v > d_hi[e], -1 if v < d_lo[e], else 0.
 * Positions p = 0..n_elements-1 (1 <= n_elements <= 128) code element
 * d_order[p] with two bits (01 = +1, 10 = -1, 00 = 0) at bit 2 (p % 16) of
 * word p / 16 of d_codes[image][k][0..7] (n_images x kp_capacity x 8
 * uint32; other bits zero); the code is 2 n_elements bits.  Rows at or
 * beyond the count are left untouched. */
cdvs_status cdvs_encode(cdvs_ctx* ctx, const cdvs_tq_model* model, int32_t n_elements, const float* d_desc,
                        const int32_t* d_count, uint32_t* d_codes, void* stream);

/* ---------------------------------------------------------------------- */
/* Global aggregation: SCFV (Sec. III-D, Eqs. (6)-(8); Sec. IV-C, Eqs. (9)-(14)) */
/* ---------------------------------------------------------------------- */
#define CDVS_SCFV_COMPONENTS 512
#define CDVS_SCFV_DIM 32

/* The aggregation model, device buffers of float32 owned by the caller:
 * PCA mean (128) and matrix (32 x 128, row r = principal direction r), and
 * a diagonal GMM of CDVS_SCFV_COMPONENTS components: weights (positive, sum
 * 1), means and variances (positive), each components x 32 row-major.  The
 * PCA mean must be 16-byte aligned. */
typedef struct {
    const float* d_pca_mean;
    const float* d_pca_matrix;
    const float* d_weights;
    const float* d_means;
    const float* d_variances;
} cdvs_scfv_model;

/* Scalable compressed Fisher vector of each image's descriptors: the first
 * d_count[image] rows of d_desc[image] (as cdvs_describe writes them:
 * n_images x kp_capacity x 128, 16-byte aligned; counts clamped to
 * 0..kp_capacity) are projected by the PCA, x_t = A (d_t - m), and
 * aggregated over the GMM: posteriors gamma_t(i) (Eq. (6)), then per
 * component i and dimension k
 *   d_gm[image][i][k] = sum_t gamma_t(i) (x_tk - mu_ik) / sigma_ik / (K sqrt(w_i))           (Eq. (7))
 *   d_gv[image][i][k] = sum_t gamma_t(i) ((x_tk - mu_ik)^2 / sigma_ik^2 - 1) / (K sqrt(2 w_i))
 * (K = the image's count; all zero when K = 0), computed in the matrix form
 * of Eqs. (10), (12), (14) on FP32 matrix cores;
 *   d_delta[image][i] = population standard deviation of d_gm[image][i][.] (Eq. (8));
 *   d_order[image][0..511] = components by delta, descending (ties: lower index
 *     first) -- the order in which a bit budget keeps them;
 *   d_bits[image][i][0], [1] = sign bits of d_gm[image][i][.] and
 *     d_gv[image][i][.], bit k set when entry k is positive.
 * Shapes: d_gm, d_gv n_images x 512 x 32 floats; d_delta n_images x 512;
 * d_order n_images x 512 int32; d_bits n_images x 512 x 2 uint32.  Uses
 * 196 KB of context scratch (so calls on one context must not overlap). */
cdvs_status cdvs_scfv(cdvs_ctx* ctx, const cdvs_scfv_model* model, const float* d_desc, const int32_t* d_count,
                      float* d_gm, float* d_gv, float* d_delta, int32_t* d_order, uint32_t* d_bits, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): cdvs_scfv without a
 * context.  It allocates nothing -- no hipMalloc, hipFree or allocating
 * library call -- and keeps its scratch in one file-scope device array of
 * CDVS_SCFV_STATIC_BYTES (8.7 MB) per GPU, held until the process ends: the
 * model's derived constants (196 KB) and 64 blocks of per-part sums
 * (130 KB each).  Its device address is looked up on the first call on each
 * device.  Batches of at most 32 images are split into parts (as many as fit
 * in the 64 blocks, at most one per 32-descriptor tile of kp_capacity); 65
 * workgroups per image add up the parts' sums and a third kernel completes
 * the image; larger batches take one workgroup per image and use only the
 * constants.  The outputs are those of cdvs_scfv (same
 * definitions, shapes and layouts; sums in another order, so equal up to
 * single-precision rounding).  d_desc is n_images x kp_capacity x 128 floats
 * (16-byte aligned), d_count n_images int32 (clamped to 0..kp_capacity).
 * Argument errors (null pointers, n_images outside 0..CDVS_MAX_IMAGES,
 * kp_capacity outside 1..CDVS_MAX_KP_CAPACITY, misalignment) return
 * CDVS_ERR_ARG before anything is enqueued, with a message from
 * cdvs_last_error(NULL) (per thread).  Every call on one GPU shares that
 * GPU's array and overwrites what it needs before reading it, so calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller. */
#define CDVS_SCFV_STATIC_BYTES 8720384
cdvs_status cdvs_scfv_noalloc(const cdvs_scfv_model* model, const float* d_desc, const int32_t* d_count,
                              int32_t n_images, int32_t kp_capacity, float* d_gm, float* d_gv, float* d_delta,
                              int32_t* d_order, uint32_t* d_bits, void* stream);

/* ---------------------------------------------------------------------- */
/* Surrogate candidate mask (a small learned CNN; not from the paper).       */
/* ---------------------------------------------------------------------- */
/* Each base image is seen as H4 x W4 cells of 4x4 pixels (H4 = ceil(H/4),
 * W4 = ceil(W/4)); cells of all images are concatenated in batch order.
 * Network: X0 = space-to-depth(4) of u8/255 (image edge-padded to a multiple
 * of 4; channel 4*dy + dx); X_l = relu(conv3x3(X_{l-1})), l = 1..4, 16
 * channels, zero padding; Z = X4 . Wh + bh, 6 logits per cell, logit o for
 * octave o.  Activations are bf16 (16 per cell, HWC); convolutions run on
 * bf16 MFMA with fp32 accumulation; the head is fp32.
 * Parameters: CDVS_CNN_PARAMS fp32 values: for l = 1..4, W_l[9][16][16]
 * ([tap][in][out], tap = 3(dy+1) + (dx+1)) then b_l[16]; then Wh[16][6]
 * ([in][octave]) and bh[6]. */
#define CDVS_CNN_PARAMS 9382
#define CDVS_CNN_CHANNELS 16
#define CDVS_CNN_HEADS 6
#define CDVS_CNN_LAYERS 4

/* Total cells of the batch, and where image `image`'s cells start. */
int64_t cdvs_cnn_cells(const cdvs_ctx* ctx);
cdvs_status cdvs_cnn_cell_layout(const cdvs_ctx* ctx, int32_t image, int64_t* cell0, int32_t* w4, int32_t* h4);

/* Forward pass on the packed u8 images.  d_acts (caller scratch, 8-byte
 * aligned): CDVS_CNN_LAYERS x cells x 16 bf16 (uint16), receives every
 * layer's output (kept for cdvs_cnn_backward); with d_acts NULL a fused
 * inference kernel keeps all activations on chip and only the outputs below
 * are written (same values).  d_logits (may be NULL): cells x 6 fp32.
 * d_mask (may be NULL): cells bytes, bit o = sigmoid(Z_o) > tau, only for
 * octaves the image has.  tau in (0, 1). */
cdvs_status cdvs_cnn_forward(cdvs_ctx* ctx, const uint8_t* d_images, const float* d_params, uint16_t* d_acts,
                             float* d_logits, uint8_t* d_mask, float tau, void* stream);

/* Training labels from detector output (e.g. cdvs_alp_detect with a large
 * topk): d_labels (cells uint32) gets bit o of the cell holding
 * (ix 2^o, iy 2^o) / 4 of every keypoint of octave o; other bits 0. */
cdvs_status cdvs_cnn_labels(cdvs_ctx* ctx, const cdvs_keypoint* d_kp, const int32_t* d_count, uint32_t* d_labels,
                            void* stream);

/* Loss and gradient for the forward pass whose d_acts / d_logits are given.
 * Loss: mean over images of each image's mean, over its cells and its
 * octaves o, of the positive-weighted cross-entropy
 * w_o y softplus(-z) + (1 - y) softplus(z), y = label bit o, w = d_pos_weight
 * (6 fp32).  d_grad (CDVS_CNN_PARAMS fp32) and d_loss (1 fp32) are
 * overwritten.  d_work: caller scratch of 2 x cells x 16 uint16. */
cdvs_status cdvs_cnn_backward(cdvs_ctx* ctx, const uint8_t* d_images, const float* d_params, const uint16_t* d_acts,
                              const float* d_logits, const uint32_t* d_labels, const float* d_pos_weight,
                              uint16_t* d_work, float* d_grad, float* d_loss, void* stream);

/* One Adam step (Kingma and Ba 2015, bias-corrected, step >= 1) on the fp32
 * parameters, with first and second moments d_m, d_v (CDVS_CNN_PARAMS each). */
cdvs_status cdvs_cnn_adam(cdvs_ctx* ctx, float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t step,
                          float lr, float beta1, float beta2, float eps, void* stream);

/* ---------------------------------------------------------------------- */
/* Streaming many batches with the host hand-off overlapped.  In the hybrid
 * encoder of Section 4 the CPU-side steps (selection, compression) run
 * concurrently with the GPU modules; here a batch of the context's shape is
 * the unit of that overlap.
 *
 * cdvs_stream processes n_chunks batches whose packed images lie at
 * d_images + c * chunk_stride (each laid out as the context's image table
 * says; chunk_stride >= the table's extent).  Per chunk, on `stream`:
 * cdvs_pyramid, then (d_cnn_params != NULL) cdvs_cnn_forward (d_acts, which
 * may be NULL) into d_mask with threshold tau and a gated cdvs_alp_detect,
 * else the plain one,
 * then cdvs_orient and cdvs_describe.  On an internal copy stream the counts,
 * oriented keypoints and descriptors are copied into pinned host slot c % 2
 * (caller-owned, from hipHostMalloc: n counts, n x kp_capacity keypoints,
 * n x kp_capacity x 128 floats per slot), and a host thread then calls
 * consumer(user, c, n, kp_capacity, counts, keypoints, descriptors) on it.
 * Chunk c + 1's pyramid, mask and detection run while chunk c is copied; a
 * slot is refilled only after the consumer returned from it.  Blocks until
 * every chunk has been consumed.  A non-zero return of the consumer stops
 * the stream (CDVS_ERR_STATE); a candidate overflow in any chunk is
 * reported as CDVS_ERR_CAPACITY at the end (results still complete). */
typedef struct {
    float* d_pyr;                 /* cdvs_pyramid_bytes */
    cdvs_keypoint* d_kp;          /* n x kp_capacity */
    int32_t* d_count;             /* n */
    cdvs_keypoint* d_kp_ori;      /* n x kp_capacity */
    int32_t* d_count_ori;         /* n */
    float* d_desc;                /* n x kp_capacity x 128 */
    const float* d_cnn_params;    /* NULL: plain detection */
    uint16_t* d_acts;             /* NULL (fused inference) or CDVS_CNN_LAYERS x cells x 16 */
    uint8_t* d_mask;              /* cells (gated only) */
    float tau;                    /* mask threshold (gated only) */
    int32_t* h_count[2];          /* pinned host double buffers */
    cdvs_keypoint* h_kp[2];
    float* h_desc[2];
} cdvs_stream_buffers;

typedef int32_t (*cdvs_chunk_consumer)(void* user, int32_t chunk, int32_t n_images, int32_t kp_capacity,
                                       const int32_t* h_count, const cdvs_keypoint* h_kp, const float* h_desc);

cdvs_status cdvs_stream(cdvs_ctx* ctx, const uint8_t* d_images, int64_t chunk_stride, int32_t n_chunks,
                        const cdvs_stream_buffers* buf, cdvs_chunk_consumer consumer, void* user, void* stream);

/* A host stand-in for the paper's CPU-side selection and compression (which
 * is not built here): a cdvs_chunk_consumer that codes every descriptor
 * element of each image's first min(count, keep) descriptors as
 * u8 = min(255, floor(512 d + 1/2)) into out[image][k][128] (image =
 * chunk * n_images + i, out laid out with kp_capacity rows per image) and
 * stores the kept count in kept[image], using `threads` host threads.
 * `user` points at a cdvs_standin_sink. */
typedef struct {
    uint8_t* out;
    int32_t* kept;
    int64_t total_images;   /* size of out / kept in images; chunks beyond it fail */
    int32_t keep;
    int32_t threads;
} cdvs_standin_sink;
int32_t cdvs_standin_consume(void* user, int32_t chunk, int32_t n_images, int32_t kp_capacity, const int32_t* h_count,
                             const cdvs_keypoint* h_kp, const float* h_desc);

/* Per-kernel timing with HIP events (tracing).  While enabled, every kernel
 * the compute calls launch is bracketed by a pair of events recorded on the
 * call's stream (so a context being captured into a graph must not have it
 * enabled).  cdvs_profile_read synchronises on the last event, adds each
 * bracket's elapsed time to total_ms[id] and launches[id] (arrays of
 * CDVS_KERNEL_COUNT entries, overwritten) and forgets the brackets.  Up to
 * 16384 brackets are kept between reads; later launches go unrecorded. */
typedef enum {
    CDVS_KERNEL_PREBLUR = 0,  /* u8 input -> G_{0,0} */
    CDVS_KERNEL_SCALES,       /* G_{o,0} -> G_{o,1..4} and G_{o+1,0}, one launch per octave */
    CDVS_KERNEL_CLEAR,        /* candidate counters */
    CDVS_KERNEL_DETECT,       /* LoG + ALP + NMS + refinement: one launch over all octaves */
    CDVS_KERNEL_FINALIZE,     /* cross-octave duplicates, sort, top-k */
    CDVS_KERNEL_ORIENT,       /* orientation histograms and peaks */
    CDVS_KERNEL_ORIENT_COMPACT,
    CDVS_KERNEL_DESCRIBE,     /* 4x4x8 descriptors */
    CDVS_KERNEL_CNN_FORWARD,  /* surrogate CNN: four convolutions and the head */
    CDVS_KERNEL_MASK_COUNT,   /* active cells of a gating mask */
    CDVS_KERNEL_SCFV,         /* SCFV aggregation (model constants + one workgroup per image) */
    CDVS_KERNEL_ENCODE,       /* transform coding and ternary quantisation */
    CDVS_KERNEL_RELEVANCE,    /* relevance scores and per-image selection */
    CDVS_KERNEL_FRONT,        /* front-end downsampling to a longer side of 640 */
    CDVS_KERNEL_BMLOG,        /* block frequency-domain scale images (one launch per octave) */
    CDVS_KERNEL_COUNT
} cdvs_kernel_id;

cdvs_status cdvs_profile_enable(cdvs_ctx* ctx, int32_t enable);
cdvs_status cdvs_profile_read(cdvs_ctx* ctx, double* total_ms, int32_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* CDVS_H */
