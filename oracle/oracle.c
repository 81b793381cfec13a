/*
 * CPU oracle for the skeleton hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct loops.  Only tests/, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the product path
 * (the HIP library) shares no code, header or table with it.
 *
 * The paper (Marrow, arXiv 1510.06585) defines the skeletons but not the
 * arithmetic of its benchmark stages; every stage below states the reading it
 * implements.  Each stage reads its whole input and writes a whole new output,
 * so a pipeline built from these functions materialises every intermediate,
 * which is the single-device depth-first execution of a skeleton tree
 * (Sec. 2, "Overview of the Marrow Algorithmic Framework").
 *
 * Images are RGBA uint8, row-major, dense: byte (y*W + x)*4 + c.
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no -ffast-math).
 * OpenMP only splits loops over independent output rows or bodies, so every
 * result is independent of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

/* ---------------------------------------------------------------------------
 * Noise stage (Sec. 4, Filter Pipeline, first filter).  The paper names a
 * "Gaussian noise" filter without parameters; the reading used here is a
 * deterministic integer hash noise: for pixel (x, y) of the stage's input and
 * seed s,
 *     key = s XOR ((y << 16) | x)              (32-bit; needs W, H <= 65536)
 *     h   = fmix32(key)                        (MurmurHash3 32-bit finaliser)
 *     n_c = ((h >> 8c) & 255) mod 33 - 16      for channel byte c = 0..3
 *     out = min(max(in + n_c, 0), 255)
 * fmix32 is written from its public description: xor-shift 16, multiply by
 * 0x85EBCA6B, xor-shift 13, multiply by 0xC2B2AE35, xor-shift 16, mod 2^32.
 * ------------------------------------------------------------------------- */
uint32_t orc_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

int orc_noise_offset(uint32_t seed, int64_t x, int64_t y, int c) {
    uint32_t key = seed ^ (((uint32_t)y << 16) | (uint32_t)x);
    uint32_t h = orc_fmix32(key);
    uint32_t b = (h >> (8 * c)) & 255u;
    return (int)(b % 33u) - 16;
}

int orc_noise(const uint8_t* in, uint8_t* out, int64_t W, int64_t H, uint32_t seed) {
    if (W < 0 || H < 0 || W > 65536 || H > 65536) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x)
            for (int c = 0; c < 4; ++c) {
                int64_t i = (y * W + x) * 4 + c;
                int v = (int)in[i] + orc_noise_offset(seed, x, y, c);
                if (v < 0) v = 0;
                if (v > 255) v = 255;
                out[i] = (uint8_t)v;
            }
    return 0;
}

/* Solarise stage (Sec. 4, Filter Pipeline, second filter): every channel byte
 * v becomes v if v < 128, else 255 - v.  Threshold 128 is the reading used. */
void orc_solarise(const uint8_t* in, uint8_t* out, int64_t nbytes) {
    for (int64_t i = 0; i < nbytes; ++i) {
        int v = in[i];
        out[i] = (uint8_t)(v < 128 ? v : 255 - v);
    }
}

/* Mirror stage (Sec. 4, Filter Pipeline, third filter).  The filters must be
 * applicable to each image line on its own (the line is the elementary
 * partitioning unit), so the mirror is left-right within a row: whole pixels
 * move, out(x, y) = in(W-1-x, y); the bytes inside a pixel keep their order. */
void orc_mirror(const uint8_t* in, uint8_t* out, int64_t W, int64_t H) {
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x)
            for (int c = 0; c < 4; ++c)
                out[(y * W + x) * 4 + c] = in[(y * W + (W - 1 - x)) * 4 + c];
}

/* 5x5 box blur stage (an added stencil Map stage; not in the paper).
 *     out(x,y,c) = floor( sum_{dy=-2..2} sum_{dx=-2..2}
 *                         in(clamp(x+dx,0,W-1), clamp(y+dy,0,H-1), c) / 25 )
 * One integer sum and one division at the end; clamp-to-edge addressing. */
static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

void orc_blur5(const uint8_t* in, uint8_t* out, int64_t W, int64_t H) {
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x)
            for (int c = 0; c < 4; ++c) {
                int64_t s = 0;
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        int64_t xx = clampi(x + dx, 0, W - 1);
                        int64_t yy = clampi(y + dy, 0, H - 1);
                        s += in[(yy * W + xx) * 4 + c];
                    }
                out[(y * W + x) * 4 + c] = (uint8_t)(s / 25);
            }
}

/* Reduce side of MapReduce (Sec. 2.1 Library; Sec. 3.4 merge by addition):
 * per channel c, hist[c*256 + v] = number of pixels whose channel c equals v
 * (uint32), and sum[c] = sum of channel c over all pixels (uint64). */
void orc_hist_sum(const uint8_t* img, int64_t W, int64_t H, uint32_t* hist, uint64_t* sum) {
    for (int i = 0; i < 4 * 256; ++i) hist[i] = 0;
    for (int c = 0; c < 4; ++c) sum[c] = 0;
    for (int64_t p = 0; p < W * H; ++p)
        for (int c = 0; c < 4; ++c) {
            uint8_t v = img[p * 4 + c];
            hist[c * 256 + v] += 1;
            sum[c] += v;
        }
}

/* Saxpy Map stage (Sec. 4, Saxpy benchmark: single-precision a*x + y).
 * Reading: one correctly rounded fp32 fused multiply-add, out = fmaf(a, v, w). */
void orc_saxpy(const float* v, const float* w, float a, float* out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) out[i] = fmaf(a, v[i], w[i]);
}

/* Mirror of a 1-D fp32 vector: out[i] = in[n-1-i]. */
void orc_reverse_f32(const float* in, float* out, int64_t n) {
    for (int64_t i = 0; i < n; ++i) out[i] = in[n - 1 - i];
}

/* fp32 sum-reduce, evaluated in fp64 over the exact fp32 values; also returns
 * sum |v_i|, the scale the tolerance is stated against. */
void orc_sum_f32(const float* v, int64_t n, double* sum, double* abs_sum) {
    double s = 0.0, a = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        s += (double)v[i];
        a += fabs((double)v[i]);
    }
    *sum = s;
    *abs_sum = a;
}

/* ---------------------------------------------------------------------------
 * N-body direct sum (Sec. 4, N-Body benchmark: every body interacts with all
 * others; the position vector is replicated whole, the COPY mode of Sec. 3.4).
 * Reading: Plummer-softened gravity in fp64,
 *     a_i = G * sum_{j=0}^{N-1} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^{3/2}
 * (the j = i term is exactly zero), then one kick-drift step
 *     v_i <- v_i + dt a_i ;  r_i <- r_i + dt v_i.
 * pos is N x 4 (x, y, z, m), vel is N x 3.
 * ------------------------------------------------------------------------- */
void orc_nbody_accel(const double* pos, double* acc, int64_t N, double G, double eps) {
    double eps2 = eps * eps;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double dx = pos[4 * j + 0] - pos[4 * i + 0];
            double dy = pos[4 * j + 1] - pos[4 * i + 1];
            double dz = pos[4 * j + 2] - pos[4 * i + 2];
            double d2 = dx * dx + dy * dy + dz * dz + eps2;
            double inv3 = 1.0 / (d2 * sqrt(d2));
            double s = pos[4 * j + 3] * inv3;
            ax += s * dx;
            ay += s * dy;
            az += s * dz;
        }
        acc[3 * i + 0] = G * ax;
        acc[3 * i + 1] = G * ay;
        acc[3 * i + 2] = G * az;
    }
}

int orc_nbody_run(double* pos, double* vel, int64_t N, int steps, double G, double eps, double dt) {
    double* acc = (double*)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
    if (!acc) return -1;
    for (int s = 0; s < steps; ++s) {
        orc_nbody_accel(pos, acc, N, G, eps);
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) {
                vel[3 * i + k] += dt * acc[3 * i + k];
                pos[4 * i + k] += dt * vel[3 * i + k];
            }
    }
    free(acc);
    return 0;
}

/* Thread count of the parallel loops (results do not depend on it). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
