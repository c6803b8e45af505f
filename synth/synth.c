/*
 * Seeded synthetic grayscale images for the CDVS front half.
 *
 * This module only makes inputs.  It holds none of the method's arithmetic
 * (no blur, no Laplacian, no fitting, no histogram): it draws a horizontal
 * intensity ramp, a set of isotropic Gaussian blobs and uniform noise, and
 * quantises to 8 bits.  Both the CPU oracle's tests and the GPU path's
 * tests/bench consume its output.
 *
 * Random numbers come from a counter-based hash built on the SplitMix64
 * output function (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014; constants as published by Vigna):
 *     sm(x)  = fmix(x + 0x9e3779b97f4a7c15)
 *     fmix(z): z ^= z >> 30; z *= 0xbf58476d1ce4e5b9;
 *              z ^= z >> 27; z *= 0x94d049bb133111eb; z ^= z >> 31
 * A draw is keyed by (seed base, image index, field, element index):
 *     h = sm(sm(sm(sm(seed) ^ image) ^ field) ^ idx)
 * and a uniform in [0,1) is the top 53 bits of h times 2^-53.
 *
 * Fields: 0 blob count, 1 blob centre x, 2 blob centre y, 3 blob scale,
 * 4 blob amplitude, 5 per-pixel noise (idx = y*W + x), 6 aspect choice.
 *
 * Pixel value, accumulated in double in a fixed order:
 *     v = 60 + 120 * x / (W-1)                         (ramp)
 *       + sum_b A_b exp(-((x-cx_b)^2 + (y-cy_b)^2) / (2 s_b^2))
 *              (each blob only within |x-cx|,|y-cy| <= ceil(4 s_b))
 *       + (2u - 1) * 8                                  (noise, u ~ U[0,1))
 *     out = clamp(floor(v + 0.5), 0, 255)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t fmix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ULL;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return z;
}

static uint64_t sm(uint64_t x) { return fmix64(x + 0x9e3779b97f4a7c15ULL); }

/* One SplitMix64 step from state x: the generator's output after x += golden. */
uint64_t synth_sm64(uint64_t x) { return sm(x); }

uint64_t synth_hash(uint64_t seed, uint64_t image, uint64_t field, uint64_t idx) {
    return sm(sm(sm(sm(seed) ^ image) ^ field) ^ idx);
}

double synth_uniform(uint64_t seed, uint64_t image, uint64_t field, uint64_t idx) {
    return (double)(synth_hash(seed, image, field, idx) >> 11) * (1.0 / 9007199254740992.0);
}

/* Blob count for image `image`: nmin + floor(u * (nmax - nmin + 1)), u from field 0. */
int synth_blob_count(uint64_t seed, uint64_t image, int nmin, int nmax) {
    if (nmax <= nmin) return nmin;
    double u = synth_uniform(seed, image, 0, 0);
    int n = nmin + (int)floor(u * (double)(nmax - nmin + 1));
    return n > nmax ? nmax : n;
}

/* Aspect choice for ragged batches: one of {4:3, 3:2, 16:9, 1:1, 3:4} with the long
 * side fixed; short side = round(long * b / a).  Writes width and height. */
void synth_aspect_size(uint64_t seed, uint64_t image, int long_side, int* width, int* height) {
    static const int num[5] = {4, 3, 16, 1, 3};
    static const int den[5] = {3, 2, 9, 1, 4};
    double u = synth_uniform(seed, image, 6, 0);
    int c = (int)floor(u * 5.0);
    if (c > 4) c = 4;
    if (num[c] >= den[c]) {
        *width = long_side;
        *height = (int)floor((double)long_side * den[c] / num[c] + 0.5);
    } else {
        *height = long_side;
        *width = (int)floor((double)long_side * num[c] / den[c] + 0.5);
    }
}

/* Render one image.  `out` has `height` rows of `pitch` bytes (pitch >= width).
 * Blob scale s ~ U[smin, smax), amplitude A ~ U[-amax, amax), centre ~ U[0,W) x U[0,H).
 * Returns 0 on success, -1 on bad arguments or allocation failure. */
int synth_image(uint64_t seed, uint64_t image, int width, int height, int pitch,
                int nblobs, double smin, double smax, double amax, uint8_t* out) {
    if (width < 2 || height < 1 || pitch < width || nblobs < 0 || !out) return -1;
    double* acc = (double*)malloc(sizeof(double) * (size_t)width * (size_t)height);
    if (!acc) return -1;
    for (int y = 0; y < height; ++y)
        for (int x = 0; x < width; ++x)
            acc[(size_t)y * width + x] = 60.0 + 120.0 * (double)x / (double)(width - 1);
    for (int b = 0; b < nblobs; ++b) {
        double cx = synth_uniform(seed, image, 1, (uint64_t)b) * width;
        double cy = synth_uniform(seed, image, 2, (uint64_t)b) * height;
        double s = smin + synth_uniform(seed, image, 3, (uint64_t)b) * (smax - smin);
        double a = (2.0 * synth_uniform(seed, image, 4, (uint64_t)b) - 1.0) * amax;
        int rad = (int)ceil(4.0 * s);
        int x0 = (int)floor(cx) - rad, x1 = (int)floor(cx) + rad + 1;
        int y0 = (int)floor(cy) - rad, y1 = (int)floor(cy) + rad + 1;
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > width - 1) x1 = width - 1;
        if (y1 > height - 1) y1 = height - 1;
        double inv = 1.0 / (2.0 * s * s);
        for (int y = y0; y <= y1; ++y) {
            double dy = (double)y - cy;
            if (fabs(dy) > rad) continue;
            for (int x = x0; x <= x1; ++x) {
                double dx = (double)x - cx;
                if (fabs(dx) > rad) continue;
                acc[(size_t)y * width + x] += a * exp(-(dx * dx + dy * dy) * inv);
            }
        }
    }
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            double u = synth_uniform(seed, image, 5, (uint64_t)y * (uint64_t)width + (uint64_t)x);
            double v = acc[(size_t)y * width + x] + (2.0 * u - 1.0) * 8.0;
            double q = floor(v + 0.5);
            if (q < 0.0) q = 0.0;
            if (q > 255.0) q = 255.0;
            out[(size_t)y * pitch + x] = (uint8_t)q;
        }
        for (int x = width; x < pitch; ++x) out[(size_t)y * pitch + x] = 0;
    }
    free(acc);
    return 0;
}
