// gfx950 kernels for batched complex fp32 FFT chains (the paper's FFT
// benchmark: FFTs of 512 KiB, i.e. 65536 complex fp32 points, pipelined
// with their inverses, Sec. 4).
//
// A 65536-point transform is computed as 256 x 256 (four-step): with
// n = n1 + 256 n2 and k = k2 + 256 k1,
//   pass A:  for every n1, a 256-point DFT over n2 -> k2, times W_N^(n1 k2),
//            stored transposed as T[k2][n1];
//   pass B:  for every k2, a 256-point DFT over n1 -> k1, giving X[k2 + 256 k1].
// Pass B of one stage and pass A of the next work on the same index (the
// next stage's n1 is this stage's k2), so a fused chain of L stages runs
// L + 1 kernels (A, L - 1 fused "BA", B) instead of 2L: the data between
// two stages never goes back to HBM.
//
// One work-group (512 threads) owns 32 columns or rows of one transform: it
// loads a 32 x 256 tile (each row of 32 elements is one 256-byte run), does
// the 256-point DFTs in LDS as 16 x 16 (a 16-point DFT per thread, a twiddle
// by W_256, a second 16-point DFT), and stores the tile the same way.
// Twiddles W_N^m are products of two roots from 256-entry LDS tables taken
// from the 65536 roots of unity computed in double precision on the host.
#include "kern_common.h"
#include "kern.h"

namespace skel {

constexpr int kFftN = kFftPoints;
constexpr int kFftR = 256;     // row / column length
constexpr int kFftCols = 32;   // rows or columns per work-group (256-byte runs)
constexpr int kFftThreads = 16 * kFftCols;   // 16 threads per 256-point DFT
// LDS tile layout: element m of row j at j * kRowStride + m + m / 16.  The
// pad after every 16 elements and the odd row stride keep both the in-row
// stride-16 reads of the DFT and the down-a-column accesses of the loads and
// stores free of bank conflicts (8-byte elements span 2 of the 32 banks).
constexpr int kRowStride = kFftR + kFftR / 16 + 1;
static __device__ __forceinline__ int sx(int j, int m) { return j * kRowStride + m + (m >> 4); }

struct cpx {
    float x, y;
};
static __device__ __forceinline__ cpx cadd(cpx a, cpx b) { return {a.x + b.x, a.y + b.y}; }
static __device__ __forceinline__ cpx csub(cpx a, cpx b) { return {a.x - b.x, a.y - b.y}; }
static __device__ __forceinline__ cpx cmul(cpx a, cpx b) {
    return {__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x)};
}
// The transform direction DIR is a template parameter: -1 forward
// (W = exp(-2 pi i / N)), +1 inverse, so no twiddle carries a run-time sign.

// a * (DIR * i)
template <int DIR>
static __device__ __forceinline__ cpx cmul_i(cpx a) { return DIR < 0 ? cpx{a.y, -a.x} : cpx{-a.y, a.x}; }

// Roots of unity in LDS: TH[h] = W^(256 h) and TL[l] = W^l (h, l < 256,
// W = exp(2 pi i / N)), so W^m = TH[m >> 8] TL[m & 255] from two reads
// instead of a scattered read of a 512 KiB table; T16[l] = W^(16 l) (l < 16)
// for the stride-16 products of the transposed stores.
struct TwLds {
    cpx hi[256], lo[256], s16[16];
};

static __device__ __forceinline__ void load_tw(TwLds& L, const float2* T) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) {
        const float2 h = T[256 * i], l = T[i];
        L.hi[i] = {h.x, h.y};
        L.lo[i] = {l.x, l.y};
        if (i < 16) {
            const float2 q = T[16 * i];
            L.s16[i] = {q.x, q.y};
        }
    }
}

// W_N^m in direction DIR: (cos, DIR * sin)(2 pi m / N), m taken mod N.
template <int DIR>
static __device__ __forceinline__ cpx tw(const TwLds& L, uint32_t m) {
    m &= (uint32_t)(kFftN - 1);
    cpx w = L.hi[m >> 8];
    if (m & 255u) w = cmul(w, L.lo[m & 255u]);
    return {w.x, DIR < 0 ? -w.y : w.y};
}

// a * W_16^K in direction DIR, the root as a compile-time constant.
template <int DIR, int K>
static __device__ __forceinline__ cpx rot16(cpx a) {
    constexpr float c8 = 0.92387953251128674f, s8 = 0.38268343236508978f, r2 = 0.70710678118654752f;
    constexpr int k = K % 16;
    if constexpr (k == 0) return a;
    else if constexpr (k == 4) return cmul_i<DIR>(a);
    else {
        constexpr float cs[16][2] = {{1, 0},   {c8, s8},   {r2, r2},   {s8, c8},   {0, 1},   {-s8, c8},
                                     {-r2, r2}, {-c8, s8}, {-1, 0},    {-c8, -s8}, {-r2, -r2}, {-s8, -c8},
                                     {0, -1},  {s8, -c8},  {r2, -r2},  {c8, -s8}};
        return cmul(a, cpx{cs[k][0], DIR < 0 ? -cs[k][1] : cs[k][1]});
    }
}

// In-register 4-point DFT of (a, b, c, d).
template <int DIR>
static __device__ __forceinline__ void dft4(cpx& a, cpx& b, cpx& c, cpx& d) {
    const cpx s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = cmul_i<DIR>(csub(b, d));
    a = cadd(s0, s1);
    c = csub(s0, s1);
    b = cadd(d0, d1);
    d = csub(d0, d1);
}

// In-register 16-point DFT, v[c] -> v[k] in natural order, as 4 x 4:
// c = c1 + 4 c2, k = k2 + 4 k1; a 4-point DFT over c2, the twiddle
// W_16^(c1 k2), a 4-point DFT over c1.
template <int DIR, int C1 = 1>
static __device__ __forceinline__ void twiddle16(cpx (&v)[16]) {
    if constexpr (C1 < 4) {
        v[C1 + 4] = rot16<DIR, C1 * 1>(v[C1 + 4]);
        v[C1 + 8] = rot16<DIR, C1 * 2>(v[C1 + 8]);
        v[C1 + 12] = rot16<DIR, C1 * 3>(v[C1 + 12]);
        twiddle16<DIR, C1 + 1>(v);
    }
}

template <int DIR>
static __device__ __forceinline__ void dft16(cpx (&v)[16]) {
#pragma unroll
    for (int c1 = 0; c1 < 4; ++c1) dft4<DIR>(v[c1], v[c1 + 4], v[c1 + 8], v[c1 + 12]);
    // v[c1 + 4 k2] now holds U[c1][k2]
    twiddle16<DIR>(v);
    cpx o[16];
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        cpx a = v[0 + 4 * k2], b = v[1 + 4 * k2], c = v[2 + 4 * k2], d = v[3 + 4 * k2];
        dft4<DIR>(a, b, c, d);
        o[k2] = a;
        o[k2 + 4] = b;
        o[k2 + 8] = c;
        o[k2 + 12] = d;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = o[k];
}

// 256-point DFTs of the kFftCols rows of a tile, thread t working on row
// j = t / 16 with u = t % 16: on entry v[c] = x[u + 16 c] of row j, on exit
// v[q] = X[u + 16 q].  The input and output element sets of a thread are the
// same, so a second transform of the same rows (the fused pass) starts from
// the registers.  S is the LDS tile used for the transposition in between;
// the call starts with a barrier (other threads may still read S) and ends
// without one.  The thread's twiddles W_256^(u p), p = 1..15, come from the
// LDS table, or with SHARED from w[p] = (cos, sin)(2 pi u p / 256): read once
// by the fused pass and used by both of its transforms.
template <int DIR, bool SHARED>
static __device__ __forceinline__ void dft256_reg(cpx* S, const TwLds& T, const cpx (&w)[16], cpx (&v)[16]) {
    const int j = threadIdx.x >> 4, u = threadIdx.x & 15;
    // m = a + 16 c with a = u: 16-point DFT over c, twiddle W_256^(a p).
    dft16<DIR>(v);
#pragma unroll
    for (int p = 1; p < 16; ++p)
        v[p] = cmul(v[p], SHARED ? cpx{w[p].x, DIR < 0 ? -w[p].y : w[p].y}
                                 : tw<DIR>(T, (uint32_t)(u * p) * (kFftN / kFftR)));
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 16; ++p) S[sx(j, 16 * p + u)] = v[p];   // Z[a = u][p] at 16 p + a
    __syncthreads();
    // for p = u: 16-point DFT over a -> k = p + 16 q
#pragma unroll
    for (int a = 0; a < 16; ++a) v[a] = S[sx(j, 16 * u + a)];
    dft16<DIR>(v);
}

template <bool SHARED>
static __device__ __forceinline__ void dft256_reg(cpx* S, const TwLds& T, const cpx (&w)[16], cpx (&v)[16],
                                                  int dir) {
    if (dir < 0)
        dft256_reg<-1, SHARED>(S, T, w, v);
    else
        dft256_reg<1, SHARED>(S, T, w, v);
}

// Twiddle W_N^(n1 k2) (n1 = kFftCols g + j, k2 = m) and store T[k2][n1].
// A thread stores one column j = t mod kFftCols at the rows m = m0 + 16 i
// (m0 = t / kFftCols, i < 16), so its twiddles are W^(n1 m0) W^(16 k) with
// k = n1 i mod 4096, and W^(16 k) = TH[k >> 4] T16[k & 15].  Across a
// wavefront these two indices are nearly consecutive or shared, so the
// reads avoid LDS bank conflicts; only W^(n1 m0) is a scattered lookup, once
// per thread.
template <int DIR>
static __device__ __forceinline__ void store_twiddled(const cpx* S, const TwLds& W, cpx* out, int g) {
    static_assert(kFftThreads % kFftCols == 0 && kFftThreads / kFftCols == 16, "one column, rows m0 + 16 i");
    const int t = threadIdx.x;
    const int j = t % kFftCols, m0 = t / kFftCols;
    const uint32_t n1 = (uint32_t)(kFftCols * g + j);
    const cpx a = tw<DIR>(W, n1 * (uint32_t)m0);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = m0 + 16 * i;
        cpx w = a;
        if (i > 0) {
            const uint32_t k = (n1 * (uint32_t)i) & 4095u;
            const cpx c = cmul(W.hi[k >> 4], W.s16[k & 15u]);
            w = cmul(a, cpx{c.x, DIR < 0 ? -c.y : c.y});
        }
        out[m * kFftTRow + kFftCols * g + j] = cmul(S[sx(j, m)], w);
    }
}

// MODE 0 (A): in natural order -> T layout; MODE 1 (BA): T -> T (pass B of
// one stage, pass A of the next); MODE 2 (B): T -> natural order.  dir1 is
// the direction of the first DFT, dir2 of the second (MODE 1); scale1 (1/N
// after an inverse stage, else 1) multiplies the result of a stage's pass B.
template <int MODE>
__global__ void __launch_bounds__(kFftThreads) fft_pass_kernel(const FftArgs A) {
    __shared__ cpx S[kFftCols * kRowStride];
    __shared__ TwLds W;
    load_tw(W, A.tw);
    const int b = blockIdx.x / (kFftR / kFftCols);
    const int g = blockIdx.x % (kFftR / kFftCols);
    const int t = threadIdx.x;
    // natural order: kFftN elements per transform; transposed (a pass A
    // output, a pass B input): 256 rows of kFftTRow
    constexpr size_t kT = (size_t)kFftR * kFftTRow;
    const cpx* in = reinterpret_cast<const cpx*>(A.in) + (size_t)b * (MODE == 0 ? (size_t)kFftN : kT);
    cpx* out = reinterpret_cast<cpx*>(A.out) + (size_t)b * (MODE == 2 ? (size_t)kFftN : kT);
    const int j = t >> 4, u = t & 15;
    cpx v[16];   // v[c] = element u + 16 c of row j of the tile
    if (MODE == 0) {
        // column n1 = kFftCols g + j, rows n2 = m: x[n1 + 256 m], staged
        // through LDS (a thread's own elements are 32-byte pieces of 16 rows)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = t + kFftThreads * i, jj = e % kFftCols, m = e / kFftCols;
            S[sx(jj, m)] = in[kFftCols * g + jj + kFftR * m];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = S[sx(j, u + 16 * c)];
    } else {
        // row k2 = kFftCols g + j of T (T[k2][m] at k2 * kFftTRow + m),
        // straight into registers: for each c the 16 threads of a row read one
        // 128-byte run
        const cpx* row = in + (size_t)(kFftCols * g + j) * kFftTRow;
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = row[u + 16 * c];
        __syncthreads();   // the twiddle tables
    }
    {
        cpx w[16];
        if (MODE == 1)
#pragma unroll
            for (int p = 1; p < 16; ++p) w[p] = W.hi[(u * p) & 255];   // W^(256 u p) = W_256^(u p)
        dft256_reg<MODE == 1>(S, W, w, v, A.dir1);
        if (MODE == 1) {
            // v[q] = X[k2 + 256 k1] of the first stage at k1 = u + 16 q (k2 =
            // kFftCols g + j): the second stage's input at n1' = k2, n2' = k1,
            // i.e. exactly what its transform of row j starts from.
            if (A.scale1 != 1.0f)
#pragma unroll
                for (int q = 0; q < 16; ++q) v[q] = {v[q].x * A.scale1, v[q].y * A.scale1};
            dft256_reg<true>(S, W, w, v, A.dir2);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) S[sx(j, u + 16 * q)] = v[q];
    }
    __syncthreads();
    if (MODE == 0 || MODE == 1) {
        if ((MODE == 0 ? A.dir1 : A.dir2) < 0)
            store_twiddled<-1>(S, W, out, g);
        else
            store_twiddled<1>(S, W, out, g);
    } else {
        // X[k2 + 256 k1] with k2 = kFftCols g + j, k1 = m
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = t + kFftThreads * i, j = e % kFftCols, m = e / kFftCols;
            const cpx v = S[sx(j, m)];
            out[kFftCols * g + j + kFftR * m] = {v.x * A.scale1, v.y * A.scale1};
        }
    }
}

hipError_t launch_fft_pass(const FftArgs& a, int mode, hipStream_t s) {
    if (a.nfft <= 0) return hipSuccess;
    const dim3 grid((unsigned)(a.nfft * (kFftR / kFftCols)));
    switch (mode) {
        case 0: hipLaunchKernelGGL(fft_pass_kernel<0>, grid, dim3(kFftThreads), 0, s, a); break;
        case 1: hipLaunchKernelGGL(fft_pass_kernel<1>, grid, dim3(kFftThreads), 0, s, a); break;
        case 2: hipLaunchKernelGGL(fft_pass_kernel<2>, grid, dim3(kFftThreads), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

const char* fft_pass_name(int mode) {
    return mode == 0 ? "fft_pass_a" : (mode == 1 ? "fft_pass_ba" : "fft_pass_b");
}

}  // namespace skel
