// gfx950 kernels for RGBA uint8 image skeletons: fused value stages (noise,
// solarise), mirror as an address remap, 5x5 box blur as a register/DPP
// sliding window, and the histogram/sum reduce side as an LDS epilogue.
//
// Work decomposition.  The paper partitions an image by lines and lets every
// work-group run the whole skeleton tree over its partition, so data passed
// between kernels never leaves the device (Sec. 3.1).  Here one wavefront owns
// a tile = a band of 256 loaded pixels (64 lanes x 4 pixels, one 16-byte load
// per lane per row) by tile_h rows, sweeps it top to bottom, and carries every
// intermediate of the fused stage chain in registers.  A blur band overlaps
// its neighbours by 2 pixels on each side (252 output pixels per band) and
// re-reads 2 rows above and below its rows; halo pixels are recomputed from
// the input, never exchanged.
//
// Packed arithmetic.  A pixel is held as two 32-bit registers of u16 pairs,
// e = {R, B} and o = {G, A}.  Noise/solarise use packed 16-bit VALU ops.  Box
// sums stay below 6375 per channel, so packed 32-bit adds never carry between
// the halves and DPP wave shifts fold the neighbour exchange into the adds.
#include "kern_common.h"
#include "kern.h"

namespace skel {

// MurmurHash3 32-bit finaliser, written from its public description.
static __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Noise on one u16 pair: b = two hash bytes; r = b mod 33 computed as
// b - 33 * ((b * 249) >> 13), exact for b in [0, 255]; out = clamp(v + r - 16).
static __device__ __forceinline__ uint32_t noise_half(uint32_t v, uint32_t hb) {
    const u16x2 b = as16(hb);
    const u16x2 q = (b * (u16x2)249) >> (u16x2)13;
    const u16x2 r = b - q * (u16x2)33;
    u16x2 t = as16(v) + r;                                   // v + n + 16 <= 287
    t = __builtin_elementwise_sub_sat(t, (u16x2)16);        // max(v + n, 0)
    t = __builtin_elementwise_min(t, (u16x2)255);
    return as32(t);
}

// Solarise on one u16 pair: min(v, 255 - v) == (v < 128 ? v : 255 - v).
static __device__ __forceinline__ uint32_t sol_half(uint32_t v) {
    const u16x2 t = as16(v);
    return as32(__builtin_elementwise_min(t, (u16x2)255 - t));
}

static __device__ __forceinline__ void noise_px(uint32_t& e, uint32_t& o, uint32_t seed, uint32_t x,
                                                uint32_t y) {
    const uint32_t h = fmix32(seed ^ ((y << 16) | x));
    e = noise_half(e, h & 0x00FF00FFu);
    o = noise_half(o, (h >> 8) & 0x00FF00FFu);
}

struct Px4 {
    uint32_t e[4], o[4];
};

// Value stages with a compile-time op sequence (ENC = sum op_k 4^k).
template <int ENC, int K>
static __device__ __forceinline__ void apply_const(const OpList& L, Px4& p, const int (&xc)[4], int y, int W) {
    if constexpr (ENC != 0) {
        constexpr int op = ENC & 3;
        if constexpr (op == IOP_NOISE) {
            const uint32_t seed = L.seed[K];
            const bool fl = L.flip[K] != 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = fl ? (W - 1 - xc[i]) : xc[i];
                noise_px(p.e[i], p.o[i], seed, (uint32_t)x, (uint32_t)y);
            }
        } else if constexpr (op == IOP_SOL) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                p.e[i] = sol_half(p.e[i]);
                p.o[i] = sol_half(p.o[i]);
            }
        }
        apply_const<(ENC >> 2), K + 1>(L, p, xc, y, W);
    }
}

template <int ENC>
static __device__ __forceinline__ void apply_ops(const OpList& L, Px4& p, const int (&xc)[4], int y, int W) {
    if constexpr (ENC == kGeneric) {
        // Stage interpreter: the op list is a kernel argument, so every branch
        // below is uniform across the wavefront.
        for (int k = 0; k < L.n; ++k) {
            const int op = L.op[k];
            if (op == IOP_NOISE) {
                const uint32_t seed = L.seed[k];
                const bool fl = L.flip[k] != 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int x = fl ? (W - 1 - xc[i]) : xc[i];
                    noise_px(p.e[i], p.o[i], seed, (uint32_t)x, (uint32_t)y);
                }
            } else if (op == IOP_SOL) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    p.e[i] = sol_half(p.e[i]);
                    p.o[i] = sol_half(p.o[i]);
                }
            }
        }
    } else {
        apply_const<ENC, 0>(L, p, xc, y, W);
    }
}

// floor(s / 25) for each u16 half, s <= 6375: (s * 5243) >> 17 is exact there.
static __device__ __forceinline__ uint32_t div25_pair(uint32_t s) {
    const uint32_t lo = s & 0xFFFFu, hi = s >> 16;
    return ((lo * 5243u) >> 17) | (((hi * 5243u) >> 17) << 16);
}

static __device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Per-tile geometry and addressing of one image.
struct ImgView {
    const uint8_t* in;
    uint8_t* out;
    int W, H;
    int in_flip, out_flip, write_out;
};

// Horizontal 5-sums of the four pixels of each lane; lane-1 and lane+1 values
// arrive through DPP wave shifts.  q[-2..5] are the 8 pixels around the lane's
// 4; t1 = q0 + q1, t2 = q2 + q3, and the left neighbour's t2 is q[-2] + q[-1].
static __device__ __forceinline__ void hsum5(const uint32_t (&q)[4], uint32_t (&h)[4]) {
    const uint32_t t1 = q[0] + q[1];
    const uint32_t t2 = q[2] + q[3];
    const uint32_t t12 = t1 + t2;
    h[0] = wave_shr1(t2) + t1 + q[2];
    h[1] = wave_shr1(q[3]) + t12;
    h[2] = wave_shl1(q[0]) + t12;
    h[3] = wave_shl1(t1) + q[1] + t2;
}

template <int PRE, int POST, bool BLUR, bool HIST>
static __device__ __forceinline__ void band_tile(const ImgView& V, const OpList& pre, const OpList& post,
                                                 int band, int y0, int y1, int lane, uint32_t* lh) {
    const int W = V.W, H = V.H;
    constexpr int halo = BLUR ? 2 : 0;
    constexpr int bw = BLUR ? kBandOut : kBandPx;
    const int x0 = band * bw;
    const int xend = min(x0 + bw, W);
    const int ub = x0 - halo + lane * 4;
    const bool interior = (x0 - halo >= 0) && (x0 - halo + kBandPx <= W);   // wave-uniform
    const uint32_t nbytes = (uint32_t)W * (uint32_t)H * 4u;
    const __amdgpu_buffer_rsrc_t rin = mk_rsrc(V.in, nbytes);
    const __amdgpu_buffer_rsrc_t rout = mk_rsrc(V.out, nbytes);

    int xc[4];
    bool valid[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        xc[i] = interior ? (ub + i) : clampi(ub + i, 0, W - 1);
        valid[i] = (ub + i >= x0) && (ub + i < xend);
    }
    const bool full = interior && valid[0] && valid[1] && valid[2] && valid[3];
    const uint32_t in_vec = (uint32_t)(V.in_flip ? (W - 4 - ub) : ub) * 4u;
    uint32_t in_px[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) in_px[i] = (uint32_t)(V.in_flip ? (W - 1 - xc[i]) : xc[i]) * 4u;
    const uint32_t out_vec = (uint32_t)(V.out_flip ? (W - 4 - ub) : ub) * 4u;

    auto load_row = [&](int yy, uint32_t (&raw)[4]) {
        const uint32_t rowoff = (uint32_t)yy * (uint32_t)W * 4u;
        if (interior) {
            const u32x4 v = ld128(rin, rowoff + in_vec);
            if (V.in_flip) {
                raw[0] = v.w; raw[1] = v.z; raw[2] = v.y; raw[3] = v.x;
            } else {
                raw[0] = v.x; raw[1] = v.y; raw[2] = v.z; raw[3] = v.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) raw[i] = ld32(rin, rowoff + in_px[i]);
        }
    };

    auto pre_px = [&](const uint32_t (&raw)[4], int yy, Px4& p) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            p.e[i] = raw[i] & 0x00FF00FFu;
            p.o[i] = (raw[i] >> 8) & 0x00FF00FFu;
        }
        apply_ops<PRE>(pre, p, xc, yy, W);
    };

    // Final pixels of one output row: store (mirrored if out_flip) and count.
    auto emit = [&](const uint32_t (&fin)[4], int y) {
        const uint32_t rowoff = (uint32_t)y * (uint32_t)W * 4u;
        if (V.write_out) {
            if (full) {
                u32x4 v;
                if (V.out_flip) {
                    v.x = fin[3]; v.y = fin[2]; v.z = fin[1]; v.w = fin[0];
                } else {
                    v.x = fin[0]; v.y = fin[1]; v.z = fin[2]; v.w = fin[3];
                }
                st128(v, rout, rowoff + out_vec);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (valid[i]) {
                        const int u = ub + i;
                        st32(fin[i], rout, rowoff + (uint32_t)(V.out_flip ? (W - 1 - u) : u) * 4u);
                    }
            }
        }
        if constexpr (HIST) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (valid[i]) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) atomicAdd(&lh[c * 256 + ((fin[i] >> (8 * c)) & 255u)], 1u);
                }
        }
    };

    if constexpr (!BLUR) {
        uint32_t nxt[4];
        load_row(y0, nxt);
        for (int y = y0; y < y1; ++y) {
            uint32_t raw[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) raw[i] = nxt[i];
            if (y + 1 < y1) load_row(y + 1, nxt);
            Px4 p;
            pre_px(raw, y, p);
            uint32_t fin[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fin[i] = p.e[i] | (p.o[i] << 8);
            emit(fin, y);
        }
    } else {
        // Sliding 5-row window of horizontal sums: ring[s] holds the row that
        // leaves the window next time slot s is visited.
        uint32_t ringE[4][4], ringO[4][4];
        uint32_t VE[4] = {0, 0, 0, 0}, VO[4] = {0, 0, 0, 0};
        auto hrow = [&](int r, uint32_t (&hE)[4], uint32_t (&hO)[4]) {
            const int rr = clampi(r, 0, H - 1);
            uint32_t raw[4];
            load_row(rr, raw);
            Px4 p;
            pre_px(raw, rr, p);
            hsum5(p.e, hE);
            hsum5(p.o, hO);
        };
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            hrow(y0 - 2 + s, ringE[s], ringO[s]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                VE[i] += ringE[s][i];
                VO[i] += ringO[s][i];
            }
        }
        uint32_t nxt[4];
        load_row(clampi(y0 + 2, 0, H - 1), nxt);
        for (int y = y0; y < y1; y += 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int yy = y + k;
                if (yy >= y1) break;
                uint32_t raw[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) raw[i] = nxt[i];
                if (yy + 1 < y1) load_row(clampi(yy + 3, 0, H - 1), nxt);
                const int rr = clampi(yy + 2, 0, H - 1);
                Px4 p;
                pre_px(raw, rr, p);
                uint32_t hE[4], hO[4];
                hsum5(p.e, hE);
                hsum5(p.o, hO);
                Px4 q;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t fe = VE[i] + hE[i];
                    const uint32_t fo = VO[i] + hO[i];
                    VE[i] = fe - ringE[k][i];
                    VO[i] = fo - ringO[k][i];
                    ringE[k][i] = hE[i];
                    ringO[k][i] = hO[i];
                    q.e[i] = div25_pair(fe);
                    q.o[i] = div25_pair(fo);
                }
                apply_ops<POST>(post, q, xc, yy, W);
                uint32_t fin[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) fin[i] = q.e[i] | (q.o[i] << 8);
                emit(fin, yy);
            }
        }
    }
}

static __device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((unsigned int)(v & 0xFFFFFFFFu), off, 64);
        const uint32_t hi = __shfl_xor((unsigned int)(v >> 32), off, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Merges an LDS histogram (4 x 256 counts) into the global histogram and
// channel sums by addition (the merge function of Sec. 3.4).  `first`/`step`
// select the bins this thread handles; lanes of one wavefront must cover
// disjoint bins.  Channel sums are derived from the counts.
static __device__ __forceinline__ void flush_hist(const uint32_t* lh, uint32_t* hist, uint64_t* sum, int first,
                                                  int step, int lane) {
    uint64_t s[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        s[c] = 0;
        for (int b = first; b < 256; b += step) {
            const uint32_t n = lh[c * 256 + b];
            if (n) {
                if (hist) atomicAdd(&hist[c * 256 + b], n);
                s[c] += (uint64_t)b * n;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint64_t t = wave_sum_u64(s[c]);
        if (lane == 0 && sum && t) atomicAdd((unsigned long long*)&sum[c], (unsigned long long)t);
    }
}

template <int PRE, int POST, bool BLUR, bool HIST>
__global__ void __launch_bounds__(256) img_band_kernel(const ImgGroupArgs A) {
    __shared__ uint32_t lh[HIST ? 1024 : 1];
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    const int wave = wave_uniform(threadIdx.x >> 6);
    if constexpr (HIST) {
        for (int b = threadIdx.x; b < 1024; b += blockDim.x) lh[b] = 0;
        __syncthreads();
    }
    const int tile = blockIdx.x * nw + wave;
    if (tile < A.ntiles) {
        const int band = tile % A.nbands;
        const int chunk = tile / A.nbands;
        const int y0 = chunk * A.tile_h;
        const int y1 = min(y0 + A.tile_h, A.H);
        const ImgView V{A.in, A.out, A.W, A.H, A.in_flip, A.out_flip, A.write_out};
        band_tile<PRE, POST, BLUR, HIST>(V, A.pre, A.post, band, y0, y1, lane, lh);
    }
    if constexpr (HIST) {
        __syncthreads();
        flush_hist(lh, A.hist, A.sum, threadIdx.x, blockDim.x, lane);
    }
}

// Persistent batched kernel: every wavefront takes tiles from a global ticket
// counter until the work list is exhausted, finds the owning request by binary
// search over the requests' first tile indices, runs the fused chain on the
// tile and merges its own LDS histogram into that request's outputs.
template <int PRE, int POST, bool BLUR, bool HIST>
__global__ void __launch_bounds__(256) img_batch_kernel(const BatchArgs A) {
    __shared__ uint32_t lh_all[HIST ? 4 * 1024 : 1];
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    uint32_t* lh = HIST ? lh_all + wave * 1024 : lh_all;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(A.counter, 1u);
        t = (uint32_t)wave_uniform((int)t);
        if (t >= (uint32_t)A.ntiles) break;
        int lo = 0, hi = A.nreq - 1;
        while (lo < hi) {   // last request with tile_begin <= t
            const int mid = (lo + hi + 1) >> 1;
            if (A.reqs[mid].tile_begin <= (int)t) lo = mid; else hi = mid - 1;
        }
        const BatchReq R = A.reqs[lo];
        const int lt = (int)t - R.tile_begin;
        const int band = lt % R.nbands;
        const int chunk = lt / R.nbands;
        const int y0 = chunk * A.tile_h;
        const int y1 = min(y0 + A.tile_h, R.H);
        if constexpr (HIST) {
            for (int b = lane; b < 1024; b += 64) lh[b] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        const ImgView V{R.in, R.out, R.W, R.H, A.in_flip, A.out_flip, 1};
        band_tile<PRE, POST, BLUR, HIST>(V, A.pre, A.post, band, y0, y1, lane, lh);
        if constexpr (HIST) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            flush_hist(lh, R.hist, R.sum, lane, 64, lane);
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Zeroes every request's histogram and sums (one work-group per request).
__global__ void batch_zero_kernel(const BatchReq* reqs, int nreq) {
    const int r = blockIdx.x;
    if (r >= nreq) return;
    const BatchReq R = reqs[r];
    for (int b = threadIdx.x; b < 1024; b += blockDim.x)
        if (R.hist) R.hist[b] = 0;
    if (threadIdx.x < 4 && R.sum) R.sum[threadIdx.x] = 0;
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------------------ host side
int encode_ops(const OpList& l) {
    int e = 0, m = 1;
    for (int k = 0; k < l.n; ++k) {
        e += m * (int)l.op[k];
        m *= 4;
    }
    return e;
}

typedef void (*img_kfn)(const ImgGroupArgs);
typedef void (*batch_kfn)(const BatchArgs);

struct ImgEntry {
    int pre, post;
    bool blur, hist;
    img_kfn fn;
    batch_kfn bfn;
    const char* name;
};

#define SKEL_IMG_ENTRY(P, Q, B, Hh, NAME) \
    {P, Q, B, Hh, img_band_kernel<P, Q, B, Hh>, img_batch_kernel<P, Q, B, Hh>, NAME}

// Specialised chains: 1 = noise, 2 = solarise, 9 = noise then solarise.
static const ImgEntry kImgTable[] = {
    SKEL_IMG_ENTRY(0, 0, false, false, "img_copy"),
    SKEL_IMG_ENTRY(1, 0, false, false, "img_noise"),
    SKEL_IMG_ENTRY(2, 0, false, false, "img_solarise"),
    SKEL_IMG_ENTRY(0, 0, false, true, "img_reduce"),
    SKEL_IMG_ENTRY(0, 0, true, false, "img_blur"),
    SKEL_IMG_ENTRY(0, 0, true, true, "img_blur_reduce"),
    SKEL_IMG_ENTRY(9, 0, false, false, "img_noise_sol"),
    SKEL_IMG_ENTRY(9, 0, false, true, "img_noise_sol_reduce"),
    SKEL_IMG_ENTRY(9, 0, true, false, "img_noise_sol_blur"),
    SKEL_IMG_ENTRY(9, 0, true, true, "img_noise_sol_blur_reduce"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, false, false, "img_generic"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, false, true, "img_generic_reduce"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, true, false, "img_generic_blur"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, true, true, "img_generic_blur_reduce"),
};

static const ImgEntry* find_entry(const OpList& pre, const OpList& post, bool blur, bool hist, int variant) {
    const int pe = encode_ops(pre), qe = encode_ops(post);
    const int n = (int)(sizeof(kImgTable) / sizeof(kImgTable[0]));
    if (variant == 0 && pre.n <= 6 && post.n <= 6) {
        for (int i = 0; i < n; ++i) {
            const ImgEntry& e = kImgTable[i];
            if (e.pre == pe && e.post == qe && e.blur == blur && e.hist == hist) return &e;
        }
    }
    for (int i = 0; i < n; ++i) {
        const ImgEntry& e = kImgTable[i];
        if (e.pre == kGeneric && e.blur == blur && e.hist == hist) return &e;
    }
    return nullptr;
}

const char* img_kernel_name(const ImgGroupArgs& a, bool blur, bool hist, int variant) {
    const ImgEntry* e = find_entry(a.pre, a.post, blur, hist, variant);
    return e ? e->name : "";
}

hipError_t launch_img_group(const ImgGroupArgs& a, bool blur, bool hist, int wg, int variant, hipStream_t s,
                            const char** kname) {
    const ImgEntry* e = find_entry(a.pre, a.post, blur, hist, variant);
    if (!e) return hipErrorInvalidValue;
    if (kname) *kname = e->name;
    if (a.ntiles <= 0) return hipSuccess;
    const int waves = wg / 64;
    const int grid = (a.ntiles + waves - 1) / waves;
    hipLaunchKernelGGL(e->fn, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_img_batch(const BatchArgs& a, int grid, int wg, hipStream_t s, const char** kname) {
    const ImgEntry* e = find_entry(a.pre, a.post, a.has_blur != 0, a.has_hist != 0, 0);
    if (!e) return hipErrorInvalidValue;
    if (kname) *kname = e->name;
    if (wg != 256 && wg != 128 && wg != 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(e->bfn, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_zero(const BatchReq* reqs, int nreq, hipStream_t s) {
    if (nreq <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_zero_kernel, dim3(nreq), dim3(256), 0, s, reqs, nreq);
    return hipGetLastError();
}

int img_batch_blocks_per_cu(const BatchArgs& a, int wg) {
    const ImgEntry* e = find_entry(a.pre, a.post, a.has_blur != 0, a.has_hist != 0, 0);
    if (!e) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(e->bfn), wg, 0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_fill_u32(void* p, uint64_t nwords, uint32_t value, hipStream_t s) {
    if (nwords == 0) return hipSuccess;
    uint64_t blocks = (nwords + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, nwords, value);
    return hipGetLastError();
}

}  // namespace skel
