// Device twin of synth.c: renders the same seeded images directly into
// device memory, for workloads too large to draw on the host in reasonable
// time (thousands of 1280x960 images).  Like synth.c it makes inputs only and
// holds none of the method's arithmetic.
//
// It follows synth.c operation for operation, in double precision with
// floating-point contraction off, so every value except exp() is computed
// with the same roundings as the host build.  exp() comes from the device
// math library, whose result can differ from the host C library's in the last
// bit; a pixel changes only if that moves v + 1/2 across an integer, which at
// ~1e-14 relative error practically never happens (the tests compare the two
// generators byte for byte).
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace {

__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ULL;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return z;
}

__device__ __forceinline__ uint64_t sm(uint64_t x) { return fmix64(x + 0x9e3779b97f4a7c15ULL); }

// sm(sm(sm(seed) ^ image) ^ field): the per-(image, field) prefix of a key
__device__ __forceinline__ uint64_t prefix(uint64_t seed, uint64_t image, uint64_t field) {
    return sm(sm(sm(seed) ^ image) ^ field);
}

__device__ __forceinline__ double unif(uint64_t pre, uint64_t idx) {
    return (double)(sm(pre ^ idx) >> 11) * (1.0 / 9007199254740992.0);
}

constexpr int kTW = 64, kTH = 16, kRows = kTH / 4;   // 256 threads, 4 rows each
constexpr int kMaxBlobs = 1536;                      // 40 B each: 60 KB of LDS

struct Blob {
    double cx, cy, a, inv;
    int rad, pad;
};

__global__ __launch_bounds__(256) void k_render(uint64_t seed, int first, int width, int height, int pitch, int nmin,
                                                int nmax, double smin, double smax, double amax, uint8_t* out,
                                                int64_t image_stride, int tiles_x, int tiles_y) {
    extern __shared__ Blob blobs[];
    const int tile = blockIdx.x % (tiles_x * tiles_y);
    const int img = blockIdx.x / (tiles_x * tiles_y);
    const uint64_t image = (uint64_t)first + (uint64_t)img;
    // blob count, as synth_blob_count
    int nb = nmin;
    if (nmax > nmin) {
        const double u = unif(prefix(seed, image, 0), 0);
        nb = nmin + (int)floor(u * (double)(nmax - nmin + 1));
        if (nb > nmax) nb = nmax;
    }
    const uint64_t p1 = prefix(seed, image, 1), p2 = prefix(seed, image, 2), p3 = prefix(seed, image, 3),
                   p4 = prefix(seed, image, 4);
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        Blob q;
        q.cx = unif(p1, (uint64_t)b) * width;
        q.cy = unif(p2, (uint64_t)b) * height;
        const double s = smin + unif(p3, (uint64_t)b) * (smax - smin);
        q.a = (2.0 * unif(p4, (uint64_t)b) - 1.0) * amax;
        q.rad = (int)ceil(4.0 * s);
        q.inv = 1.0 / (2.0 * s * s);
        q.pad = 0;
        blobs[b] = q;
    }
    __syncthreads();

    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x = tx * kTW + (threadIdx.x % kTW);
    const int y0 = ty * kTH + (threadIdx.x / kTW) * kRows;
    const double ramp = 60.0 + 120.0 * (double)x / (double)(width - 1);
    double acc[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) acc[r] = ramp;
    const double tx0 = tx * kTW, tx1 = tx * kTW + kTW - 1, ty0 = ty * kTH, ty1 = ty * kTH + kTH - 1;
    for (int b = 0; b < nb; ++b) {
        const Blob q = blobs[b];
        // skip blobs whose square window misses the whole tile (uniform branch)
        // (one pixel of slack, so rounding here never drops a blob the exact test below keeps)
        if (q.cx + (q.rad + 1) < tx0 || q.cx - (q.rad + 1) > tx1 || q.cy + (q.rad + 1) < ty0 ||
            q.cy - (q.rad + 1) > ty1)
            continue;
        const double dx = (double)x - q.cx;
        if (fabs(dx) > q.rad) continue;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const double dy = (double)(y0 + r) - q.cy;
            if (fabs(dy) <= q.rad) acc[r] += q.a * exp(-(dx * dx + dy * dy) * q.inv);
        }
    }
    uint8_t* dst = out + (int64_t)img * image_stride;
    const uint64_t p5 = prefix(seed, image, 5);
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int y = y0 + r;
        if (y >= height || x >= pitch) continue;
        uint8_t v8 = 0;
        if (x < width) {
            const double u = unif(p5, (uint64_t)y * (uint64_t)width + (uint64_t)x);
            const double v = acc[r] + (2.0 * u - 1.0) * 8.0;
            double q = floor(v + 0.5);
            if (q < 0.0) q = 0.0;
            if (q > 255.0) q = 255.0;
            v8 = (uint8_t)q;
        }
        dst[(int64_t)y * pitch + x] = v8;
    }
}

}  // namespace

extern "C" {

// Renders images first .. first+n-1 of seed base `seed`, all width x height,
// image i at d_out + i * image_stride, rows of `pitch` bytes (bytes past the
// width are zeroed).  Blob count per image from U{nmin..nmax} as
// synth_blob_count (nmin == nmax: exactly nmin; at most 1536).  Asynchronous
// on `stream`.
// Returns 0, -1 on bad arguments, -2 on a launch error.
int synth_dev_batch(uint64_t seed, int first, int n, int width, int height, int pitch, int nmin, int nmax,
                    double smin, double smax, double amax, uint8_t* d_out, int64_t image_stride, void* stream) {
    if (width < 2 || height < 1 || pitch < width || n < 0 || first < 0 || nmin < 0 || nmax < 0 || !d_out ||
        image_stride < (int64_t)pitch * height)
        return -1;
    const int nbmax = nmax > nmin ? nmax : nmin;
    if (nbmax > kMaxBlobs) return -1;   // the blob table lives in LDS
    if (n == 0) return 0;
    const int tiles_x = (pitch + kTW - 1) / kTW, tiles_y = (height + kTH - 1) / kTH;
    const int64_t blocks = (int64_t)n * tiles_x * tiles_y;
    if (blocks > 0x7fffffff) return -1;
    const size_t lds = sizeof(Blob) * (size_t)(nbmax > 0 ? nbmax : 1);
    hipLaunchKernelGGL(k_render, dim3((unsigned)blocks), dim3(256), lds, (hipStream_t)stream, seed, first, width,
                       height, pitch, nmin, nmax, smin, smax, amax, d_out, image_stride, tiles_x, tiles_y);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
