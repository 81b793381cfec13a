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
#include <hip/hip_ext.h>

#include "kern_common.h"
#include "kern.h"

#include <algorithm>
#include <type_traits>

namespace skel {

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

// Noise followed by solarise on one u16 pair.  With t = v + n, n in [-16, 16],
// solarise(clamp(t, 0, 255)) == max(0, min(t, 255 - t)) for every t in
// [-16, 271]; in unsigned form with t' = t + 16 that is
// min(sat(t' - 16), sat(271 - t')), three packed ops instead of four.
static __device__ __forceinline__ uint32_t noise_sol_half(uint32_t v, uint32_t hb) {
    const u16x2 b = as16(hb);
    const u16x2 q = (b * (u16x2)249) >> (u16x2)13;
    const u16x2 t = as16(v) + (b - q * (u16x2)33);          // t' = v + n + 16 in [0, 287]
    const u16x2 lo = __builtin_elementwise_sub_sat(t, (u16x2)16);
    const u16x2 hi = __builtin_elementwise_sub_sat((u16x2)271, t);
    return as32(__builtin_elementwise_min(lo, hi));
}

// Bytes 1 and 3 of v as a u16 pair (bytes 0 and 2 are v & 0x00FF00FF).
static __device__ __forceinline__ uint32_t odd_bytes(uint32_t v) {
    return __builtin_amdgcn_perm(0u, v, 0x0C030C01u);
}

// h ^ (h >> 16) as one SDWA instruction: the low half becomes lo ^ hi and
// the high half is kept (it is xored with zero).
static __device__ __forceinline__ uint32_t xor_hi_into_lo(uint32_t h) {
    uint32_t r = h;
    asm("v_xor_b32_sdwa %0, %1, %1 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:WORD_1 src1_sel:WORD_0"
        : "+v"(r)
        : "v"(h));
    return r;
}

// The MurmurHash3 32-bit finaliser (written from its public description) of
// the key seed ^ ((y << 16) | x), x < 2^16.  The key's high half does not
// depend on x, so the finaliser's first xor-shift k ^ (k >> 16) equals
// (S ^ (S >> 16)) ^ x with S = seed ^ (y << 16), a wavefront-uniform value.
static __device__ __forceinline__ uint32_t px_hash(uint32_t seed, uint32_t x, uint32_t y) {
    const uint32_t S = seed ^ (y << 16);
    uint32_t h = (S ^ (S >> 16)) ^ x;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    return xor_hi_into_lo(h);
}

static __device__ __forceinline__ void noise_px(uint32_t& e, uint32_t& o, uint32_t seed, uint32_t x,
                                                uint32_t y) {
    const uint32_t h = px_hash(seed, x, y);
    e = noise_half(e, h & 0x00FF00FFu);
    o = noise_half(o, odd_bytes(h));
}

static __device__ __forceinline__ void noise_sol_px(uint32_t& e, uint32_t& o, uint32_t seed, uint32_t x,
                                                    uint32_t y) {
    const uint32_t h = px_hash(seed, x, y);
    e = noise_sol_half(e, h & 0x00FF00FFu);
    o = noise_sol_half(o, odd_bytes(h));
}

struct Px4 {
    uint32_t e[4], o[4];
};

// Value stages with a compile-time op sequence (ENC = sum op_k 4^k).
template <int ENC, int K>
static __device__ __forceinline__ void apply_const(const OpList& L, Px4& p, const int (&xc)[4], int y, int W) {
    if constexpr (ENC != 0) {
        constexpr int op = ENC & 3;
        if constexpr (op == IOP_NOISE && ((ENC >> 2) & 3) == IOP_SOL) {
            const uint32_t seed = L.seed[K];
            const bool fl = L.flip[K] != 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = fl ? (W - 1 - xc[i]) : xc[i];
                noise_sol_px(p.e[i], p.o[i], seed, (uint32_t)x, (uint32_t)y);
            }
            apply_const<(ENC >> 4), K + 2>(L, p, xc, y, W);
            return;
        } else if constexpr (op == IOP_NOISE) {
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
            if (op == IOP_NOISE && k + 1 < L.n && L.op[k + 1] == IOP_SOL) {
                const uint32_t seed = L.seed[k];
                const bool fl = L.flip[k] != 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int x = fl ? (W - 1 - xc[i]) : xc[i];
                    noise_sol_px(p.e[i], p.o[i], seed, (uint32_t)x, (uint32_t)y);
                }
                ++k;
            } else if (op == IOP_NOISE) {
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

// floor(s / 25) for each u16 half, s <= 6375: (s * 671089) >> 24 is exact
// there and the product fits 32 bits, so each quotient lands in byte 3 of a
// 24-bit multiply and one byte permute gathers both into a u16 pair.
static __device__ __forceinline__ uint32_t div25_pair(uint32_t s) {
    const uint32_t mlo = (s & 0xFFFFu) * 671089u, mhi = (s >> 16) * 671089u;
    return __builtin_amdgcn_perm(mhi, mlo, 0x0C070C03u);
}

static __device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Input rows in flight per wavefront ahead of the row being computed
// (pointwise chains; a blur keeps one per slot of its 5-row ring).
constexpr int kPrefetch = 4;
static_assert(kPrefetch == 4, "pointwise row groups are written out for four slots");
constexpr int kBlurRing = 5;
static_assert(kBlurRing == 5, "blur row groups are written out for five slots");

// Histogram modes: none, or one privatised histogram per work-group with
// kHistWgChan counter words = bins x copies per channel.  HIST_WG: counter
// (c, v, copy) at word c * kHistWgChan + v * copies + copy.  HIST_WG128
// (128 bins, 16 copies): at word v * 64 + c * 16 + copy, i.e. byte address
// v * 256 + c * 64 + 4 * copy, which one byte permute builds from the value
// byte and the lane's copy offset (c * 64 is the instruction's offset).
enum { HIST_NONE = 0, HIST_WG = 1, HIST_WG128 = 2 };
constexpr int kHistWgChan = 2048;

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

template <int PRE, int POST, bool BLUR, int HM>
static __device__ __forceinline__ void band_tile(const ImgView& V, const OpList& pre, const OpList& post,
                                                 int band, int y0, int y1, int lane, uint32_t* lh, int hks) {
    constexpr bool HIST = HM != HIST_NONE;
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

    // Histogram addressing: counter (c, v, copy) lives at word
    // c * CS + v * 2^hks + copy, copy = lane mod 2^hks; a u16 pair {v0, v1}
    // shifted left by hks + 2 gives both byte offsets in its halves.
    constexpr int CS = kHistWgChan;
    const uint32_t hsh = (uint32_t)hks + 2u;
    const uint32_t lane_off = ((uint32_t)lane & ((1u << hks) - 1u)) * 4u;
    char* const lhb = reinterpret_cast<char*>(lh);
    auto count = [&](uint32_t e, uint32_t o, uint32_t inc) {
        if constexpr (HM == HIST_WG128) {
            // byte 1 of the address = the value, byte 0 = the copy offset
            // (< 64), bytes 2-3 = 0; channels R, G, B, A at offsets 0, 64,
            // 128, 192 (e = {R, B}, o = {G, A})
            const uint32_t aR = __builtin_amdgcn_perm(e, lane_off, 0x0C0C0400u);
            const uint32_t aB = __builtin_amdgcn_perm(e, lane_off, 0x0C0C0600u);
            const uint32_t aG = __builtin_amdgcn_perm(o, lane_off, 0x0C0C0400u);
            const uint32_t aA = __builtin_amdgcn_perm(o, lane_off, 0x0C0C0600u);
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + aR), inc);
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + 64 + aG), inc);
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + 128 + aB), inc);
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + 192 + aA), inc);
        } else {
            const uint32_t es = e << hsh, os = o << hsh;
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + 0 * CS * 4 + lane_off + (es & 0xFFFFu)), inc);
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + 1 * CS * 4 + lane_off + (os & 0xFFFFu)), inc);
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + 2 * CS * 4 + lane_off + (es >> 16)), inc);
            atomicAdd(reinterpret_cast<uint32_t*>(lhb + 3 * CS * 4 + lane_off + (os >> 16)), inc);
        }
    };

    // The row sweep, instantiated once for interior bands (one 16-byte load
    // and store per lane per row) and once for bands touching the image edge
    // (clamped per-pixel loads, per-pixel stores).  Prefetched rows stay raw
    // until consumed, so no load result is touched before its row's turn.
    auto sweep = [&](auto interior_tag) {
        constexpr bool I = decltype(interior_tag)::value;
        int xc[4];
        bool valid[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            xc[i] = I ? (ub + i) : clampi(ub + i, 0, W - 1);
            valid[i] = (ub + i >= x0) && (ub + i < xend);
        }
        const bool full = I && valid[0] && valid[1] && valid[2] && valid[3];
        // Interior blur bands: lane 0 owns output pixels 2..3 of its four and
        // lane 63 pixels 0..1; each writes its pair with one 8-byte store.
        const int pair0 = valid[0] ? 0 : 2;
        const bool pair = I && !full && (valid[0] || valid[2]);
        const uint32_t pair_off =
            (uint32_t)(V.out_flip ? (W - 2 - (ub + pair0)) : (ub + pair0)) * 4u;
        uint32_t inc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) inc[i] = valid[i] ? 1u : 0u;
        const uint32_t in_vec = (uint32_t)(V.in_flip ? (W - 4 - ub) : ub) * 4u;
        uint32_t in_px[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) in_px[i] = (uint32_t)(V.in_flip ? (W - 1 - xc[i]) : xc[i]) * 4u;
        const uint32_t out_vec = (uint32_t)(V.out_flip ? (W - 4 - ub) : ub) * 4u;

        auto load_row = [&](int yy) -> u32x4 {
            const uint32_t rowoff = (uint32_t)yy * (uint32_t)W * 4u;
            if constexpr (I) {
                return ld128(rin, rowoff + in_vec);
            } else {
                u32x4 r;
                r.x = ld32(rin, rowoff + in_px[0]);
                r.y = ld32(rin, rowoff + in_px[1]);
                r.z = ld32(rin, rowoff + in_px[2]);
                r.w = ld32(rin, rowoff + in_px[3]);
                return r;
            }
        };

        // Pixels of a loaded row in iteration order, split into channel pairs.
        auto unpack = [&](const u32x4& v, Px4& p) {
            uint32_t raw[4];
            if (I && V.in_flip) {
                raw[0] = v.w; raw[1] = v.z; raw[2] = v.y; raw[3] = v.x;
            } else {
                raw[0] = v.x; raw[1] = v.y; raw[2] = v.z; raw[3] = v.w;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                p.e[i] = raw[i] & 0x00FF00FFu;
                p.o[i] = odd_bytes(raw[i]);
            }
        };

        // Final pixels of one output row (e/o = their channel pairs): store
        // (mirrored if out_flip) and count.
        auto emit = [&](const Px4& q, int y) {
            uint32_t fin[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fin[i] = q.e[i] | (q.o[i] << 8);
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
                } else if (I) {
                    // In an interior band every lane is full except the two
                    // halo lanes of a stencil band, which store a pair.
                    const uint32_t a = pair0 ? fin[2] : fin[0];
                    const uint32_t b = pair0 ? fin[3] : fin[1];
                    u32x2 v;
                    v.x = V.out_flip ? b : a;
                    v.y = V.out_flip ? a : b;
                    if (pair) st64(v, rout, rowoff + pair_off);
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
                // Invalid pixels add 0: no branch on per-lane validity.
#pragma unroll
                for (int i = 0; i < 4; ++i) count(q.e[i], q.o[i], inc[i]);
            }
        };

        if constexpr (!BLUR) {
            // Rows are prefetched kPrefetch ahead; slot k is refilled as soon
            // as it is consumed (refills are clamped to the tile, so the last
            // rows re-read cached lines).  Whole groups of kPrefetch rows run
            // in a loop with no early exit and the last y1 - y0 mod kPrefetch
            // rows after it, so the loop back-edge only waits for the oldest
            // row in flight.
            u32x4 nxt[kPrefetch];
#pragma unroll
            for (int d = 0; d < kPrefetch; ++d) nxt[d] = load_row(min(y0 + d, y1 - 1));
            auto row = [&](auto kc, int yy, bool refill) {
                constexpr int k = decltype(kc)::value;
                Px4 p;
                unpack(nxt[k], p);                                              // slot consumed ...
                if (refill) nxt[k] = load_row(min(yy + kPrefetch, y1 - 1));     // ... and refilled
                apply_ops<PRE>(pre, p, xc, yy, W);
                emit(p, yy);
            };
            int y = y0;
            for (; y + kPrefetch <= y1; y += kPrefetch) {
                row(std::integral_constant<int, 0>{}, y, true);
                row(std::integral_constant<int, 1>{}, y + 1, true);
                row(std::integral_constant<int, 2>{}, y + 2, true);
                row(std::integral_constant<int, 3>{}, y + 3, true);
            }
            const int rem = y1 - y;
            if (rem > 0) row(std::integral_constant<int, 0>{}, y, false);
            if (rem > 1) row(std::integral_constant<int, 1>{}, y + 1, false);
            if (rem > 2) row(std::integral_constant<int, 2>{}, y + 2, false);
        } else {
            // Sliding 5-row window of horizontal sums in a ring of 5 slots,
            // one per row of the window: the row entering the window goes to
            // the slot of the row that left it one output row earlier, so no
            // slot's old and new values are live at once and the loop carries
            // every slot in place.  Rows are numbered from y0 - 2: slots 0-3
            // start with rows y0 - 2 .. y0 + 1; output row y0 + t adds row
            // t + 4 (slot (t + 4) mod 5) and then drops row t (slot t mod 5).
            constexpr int R = kBlurRing;
            uint32_t ringE[R][4], ringO[R][4];
            uint32_t VE[4] = {0, 0, 0, 0}, VO[4] = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int rr = clampi(y0 - 2 + s, 0, H - 1);
                Px4 p;
                unpack(load_row(rr), p);
                apply_ops<PRE>(pre, p, xc, rr, W);
                hsum5(p.e, ringE[s]);
                hsum5(p.o, ringO[s]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    VE[i] += ringE[s][i];
                    VO[i] += ringO[s][i];
                }
            }
            // Input rows y+2 ... are prefetched R ahead (one slot per row of
            // an unrolled group, so every slot index is a constant); refills
            // are clamped to the last row the tile needs, y1 + 1.  As above,
            // whole groups of R rows loop with no early exit.
            const int last = min(y1 + 1, H - 1);
            u32x4 nxt[R];
#pragma unroll
            for (int d = 0; d < R; ++d) nxt[d] = load_row(min(y0 + 2 + d, last));
            auto row = [&](auto kc, int yy, bool refill) {
                constexpr int j = decltype(kc)::value;      // (yy - y0) mod R
                constexpr int sn = (j + 4) % R;             // slot of the entering row
                const int rr = min(yy + 2, H - 1);
                Px4 p;
                unpack(nxt[j], p);                                                // slot consumed ...
                if (refill) nxt[j] = load_row(min(yy + 2 + R, last));             // ... and refilled
                apply_ops<PRE>(pre, p, xc, rr, W);
                hsum5(p.e, ringE[sn]);
                hsum5(p.o, ringO[sn]);
                Px4 q;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t fe = VE[i] + ringE[sn][i];
                    const uint32_t fo = VO[i] + ringO[sn][i];
                    VE[i] = fe - ringE[j][i];
                    VO[i] = fo - ringO[j][i];
                    q.e[i] = div25_pair(fe);
                    q.o[i] = div25_pair(fo);
                }
                apply_ops<POST>(post, q, xc, yy, W);
                emit(q, yy);
            };
            int y = y0;
            for (; y + R <= y1; y += R) {
                row(std::integral_constant<int, 0>{}, y, true);
                row(std::integral_constant<int, 1>{}, y + 1, true);
                row(std::integral_constant<int, 2>{}, y + 2, true);
                row(std::integral_constant<int, 3>{}, y + 3, true);
                row(std::integral_constant<int, 4>{}, y + 4, true);
            }
            const int rem = y1 - y;
            if (rem > 0) row(std::integral_constant<int, 0>{}, y, false);
            if (rem > 1) row(std::integral_constant<int, 1>{}, y + 1, false);
            if (rem > 2) row(std::integral_constant<int, 2>{}, y + 2, false);
            if (rem > 3) row(std::integral_constant<int, 3>{}, y + 3, false);
        }
    };
    if (interior)
        sweep(std::true_type{});
    else
        sweep(std::false_type{});
}

// Sums the 2^hks copies of every counter of a privatised LDS histogram and
// stores the counts as one row of 4 x bins words (channel-major) with plain
// stores; threads [first, first + step) cover the row.  The rows are merged by
// the histogram finalise kernels, so no device-wide atomics are needed.
// Counter (c, v, copy) is at word c * CS + v * 2^hks + copy; thread order
// starts each bin's copy sum at a different copy to spread LDS banks.
// With CLEAR every counter is zeroed after it is read (each word is read by
// one thread only), leaving the histogram ready for the next tile group.
template <int CS, bool CLEAR = false, bool L128 = false>
static __device__ __forceinline__ void write_hist_row(uint32_t* lh, int hks, uint32_t* row, int first, int step) {
    const int copies = 1 << hks;
    const int bins = CS >> hks;
    for (int b = first; b < 4 * bins; b += step) {
        const int c = b >> (__builtin_ctz((unsigned)bins));
        const int v = b & (bins - 1);
        uint32_t* w = L128 ? lh + v * 64 + c * 16 : lh + c * CS + (v << hks);
        uint32_t n = 0;
        for (int j = 0; j < copies; ++j) {
            n += w[(j + v) & (copies - 1)];
            if (CLEAR) w[(j + v) & (copies - 1)] = 0;
        }
        row[b] = n;
    }
}

// FL >= 0 fixes the mirror flags at compile time (bit 0: input, bit 1:
// output), which removes the per-row selects of the flipped data order;
// FL = -1 reads them from the arguments.
template <int PRE, int POST, bool BLUR, bool HIST, int FL>
__global__ void __launch_bounds__(256) img_band_kernel(const ImgGroupArgs A) {
    __shared__ uint32_t lh[HIST ? 4 * kHistWgChan : 1];
    if (A.guard && *A.guard == 0) return;   // a finished while Loop: the whole grid returns
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    const int wave = wave_uniform(threadIdx.x >> 6);
    if constexpr (HIST) {
        // Work-group 0 clears the reduce outputs; the merge kernel that runs
        // after this launch adds the work-groups' histogram rows to them.
        if (blockIdx.x == 0) {
            for (int b = threadIdx.x; b < 1024; b += blockDim.x)
                if (A.hist) A.hist[b] = 0;
            if (threadIdx.x < 4 && A.sum) A.sum[threadIdx.x] = 0;
        }
        for (int b = threadIdx.x; b < 4 * kHistWgChan; b += blockDim.x) lh[b] = 0;
        __syncthreads();
    }
    const int tile = blockIdx.x * nw + wave;
    if (tile < A.ntiles) {
        const int band = tile % A.nbands;
        const int chunk = tile / A.nbands;
        const int y0 = chunk * A.tile_h;
        const int y1 = min(y0 + A.tile_h, A.H);
        const ImgView V{A.in, A.out, A.W, A.H, FL < 0 ? A.in_flip : (FL & 1), FL < 0 ? A.out_flip : (FL >> 1),
                        A.write_out};
        if (HIST && A.bins == 128)
            band_tile<PRE, POST, BLUR, HIST ? HIST_WG128 : HIST_NONE>(V, A.pre, A.post, band, y0, y1, lane, lh,
                                                                       A.hist_ks);
        else
            band_tile<PRE, POST, BLUR, HIST ? HIST_WG : HIST_NONE>(V, A.pre, A.post, band, y0, y1, lane, lh,
                                                                    A.hist_ks);
    }
    if constexpr (HIST) {
        __syncthreads();
        if (A.bins == 128)
            write_hist_row<kHistWgChan, false, true>(lh, A.hist_ks, A.part + (size_t)blockIdx.x * 4 * A.bins,
                                                     threadIdx.x, blockDim.x);
        else
            write_hist_row<kHistWgChan>(lh, A.hist_ks, A.part + (size_t)blockIdx.x * 4 * A.bins, threadIdx.x,
                                        blockDim.x);
    }
}

// A request descriptor read into scalar registers word by word: every lane
// loads the same address, and without the read-back the pointers and sizes
// would stay in vector registers, turning all of the tile's addressing into
// per-lane arithmetic.
static __device__ __forceinline__ BatchReq uniform_req(const BatchReq* p) {
    static_assert(sizeof(BatchReq) % 4 == 0, "descriptor is whole words");
    BatchReq r;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(BatchReq) / 4); ++i) dst[i] = (uint32_t)wave_uniform((int)src[i]);
    return r;
}

// Persistent batched kernel: every work-group takes a group of consecutive
// tiles (one per wavefront: adjacent bands of the same rows, so the group
// streams contiguous row segments through one CU's cache, as a work-group of
// the single-image kernel does) from a global ticket counter until the work
// list is exhausted.  The host pads every request's tiles to whole groups, so
// a group never spans two requests: its wavefronts count into one
// work-group histogram, stored as the group's histogram row (row = ticket).
// Each wavefront looks up its tile's request in the tile -> request table;
// padding tiles (past the request's last tile) do nothing.
template <int PRE, int POST, bool BLUR, bool HIST, int FL>
__global__ void __launch_bounds__(256) img_batch_kernel(const BatchArgs A) {
    __shared__ uint32_t lh[HIST ? 4 * kHistWgChan : 1];
    __shared__ uint32_t ticket[2];
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const uint32_t nw = blockDim.x >> 6;
    if constexpr (HIST)
        for (int b = threadIdx.x; b < 4 * kHistWgChan; b += blockDim.x) lh[b] = 0;
    // ticket[] alternates between iterations: thread 0 writes slot i & 1 only
    // after the barrier of iteration i - 1, which every wavefront reaches
    // after reading the same slot in iteration i - 2.  That barrier also
    // orders the previous group's histogram read-and-clear before new counts.
    for (uint32_t it = 0;; ++it) {
        if (threadIdx.x == 0) ticket[it & 1] = atomicAdd(A.counter, 1u);
        __syncthreads();
        const uint32_t g = (uint32_t)wave_uniform((int)ticket[it & 1]);
        if (g * nw >= (uint32_t)A.ntiles) break;   // uniform over the work-group
        const uint32_t t = g * nw + (uint32_t)wave;
        const BatchReq R = uniform_req(A.reqs + wave_uniform((int)A.tile_req[t]));
        const int lt = (int)t - R.tile_begin;
        if (lt < R.nbands * R.nchunks) {
            const int band = lt % R.nbands;
            const int chunk = lt / R.nbands;
            const int y0 = chunk * R.tile_h;
            const int y1 = min(y0 + R.tile_h, R.H);
            const ImgView V{R.in, R.out, R.W, R.H, FL < 0 ? A.in_flip : (FL & 1), FL < 0 ? A.out_flip : (FL >> 1),
                            1};
            if (HIST && A.bins == 128)
                band_tile<PRE, POST, BLUR, HIST ? HIST_WG128 : HIST_NONE>(V, A.pre, A.post, band, y0, y1, lane, lh,
                                                                           A.hist_ks);
            else
                band_tile<PRE, POST, BLUR, HIST ? HIST_WG : HIST_NONE>(V, A.pre, A.post, band, y0, y1, lane, lh,
                                                                        A.hist_ks);
        }
        if constexpr (HIST) {
            __syncthreads();
            if (A.bins == 128)
                write_hist_row<kHistWgChan, true, true>(lh, A.hist_ks, A.part + (size_t)g * 4 * A.bins, threadIdx.x,
                                                        blockDim.x);
            else
                write_hist_row<kHistWgChan, true>(lh, A.hist_ks, A.part + (size_t)g * 4 * A.bins, threadIdx.x,
                                                  blockDim.x);
        }
    }
}

static __device__ __forceinline__ u32x4 ldg128(const uint32_t* p) { return *reinterpret_cast<const u32x4*>(p); }

static __device__ __forceinline__ int seg_of(const HistFinArgs& F, int chunk) {
    if (!F.segs) return 0;
    int lo = 0, hi = F.nseg - 1;
    while (lo < hi) {   // last segment with chunk_begin <= chunk
        const int mid = (lo + hi + 1) >> 1;
        if (F.segs[mid].chunk_begin <= chunk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sum of rows [0, nrows) (stride `words`) of `base` by a 1024-thread work-
// group: thread (g, q), g < G = 4096 / words, sums the 16-byte word group q of
// rows g, g + G, ... with kSumUnroll loads in flight, and the G partial sums
// of q meet in LDS.  Threads with g == 0 return the total of their q.
constexpr int kFinThreads = 1024;
constexpr int kSumUnroll = 8;
static __device__ __forceinline__ u32x4 sum_rows(const uint32_t* base, int nrows, int words, u32x4* red) {
    const int nq = words >> 2;
    const int G = kFinThreads / nq;
    const int q = threadIdx.x % nq, g = threadIdx.x / nq;
    u32x4 acc[kSumUnroll];
#pragma unroll
    for (int u = 0; u < kSumUnroll; ++u) acc[u] = u32x4{0, 0, 0, 0};
    for (int r0 = g; r0 < nrows; r0 += kSumUnroll * G) {
        u32x4 v[kSumUnroll];
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) {
            const int r = r0 + u * G;
            v[u] = r < nrows ? ldg128(base + (size_t)r * words + 4 * q) : u32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) acc[u] += v[u];
    }
#pragma unroll
    for (int u = 1; u < kSumUnroll; ++u) acc[0] += acc[u];
    __syncthreads();   // red may still be read by a previous call
    red[threadIdx.x] = acc[0];
    __syncthreads();
    u32x4 t = u32x4{0, 0, 0, 0};
    if (g == 0)
        for (int k = 0; k < G; ++k) t += red[k * nq + q];
    return t;
}

// Merge (one launch after the kernels that wrote the rows): work-group k sums
// the rows of chunk k.  A segment of one chunk gets its outputs written with
// plain stores; the chunks of a longer segment add their non-zero counts, and
// the channel sums they imply, to its outputs with device-scope atomics, the
// outputs having been cleared before the rows were written (by
// hist_zero_kernel or by work-group 0 of the image kernel).
__global__ void __launch_bounds__(kFinThreads) hist_merge_kernel(const HistFinArgs F) {
    __shared__ u32x4 red[kFinThreads];
    __shared__ unsigned long long csum[4];
    if (F.guard && *F.guard == 0) return;
    const int k = blockIdx.x;
    const HistSeg& S = F.segs ? F.segs[seg_of(F, k)] : F.one;
    const int words = 4 * F.bins;
    const int r0 = S.row_begin + (k - S.chunk_begin) * S.crows;
    const int r1 = min(r0 + S.crows, S.row_begin + S.nrows);
    const bool direct = S.nrows <= S.crows;
    if (threadIdx.x < 4) csum[threadIdx.x] = 0;
    const u32x4 n = sum_rows(F.part + (size_t)r0 * words, max(r1 - r0, 0), words, red);
    if ((int)threadIdx.x < (words >> 2)) {
        const int b = 4 * threadIdx.x;
        const int c = b >> __builtin_ctz((unsigned)F.bins), v = b & (F.bins - 1);
        if (S.hist) {
            uint32_t* h = S.hist + c * 256 + v;
            if (direct) {
                *reinterpret_cast<u32x4*>(h) = n;
            } else {
                if (n.x) atomicAdd(h, n.x);
                if (n.y) atomicAdd(h + 1, n.y);
                if (n.z) atomicAdd(h + 2, n.z);
                if (n.w) atomicAdd(h + 3, n.w);
            }
        }
        const unsigned long long t = (unsigned long long)v * n.x + (unsigned long long)(v + 1) * n.y +
                                     (unsigned long long)(v + 2) * n.z + (unsigned long long)(v + 3) * n.w;
        if (t) atomicAdd(&csum[c], t);
    }
    const int per = 256 - F.bins;
    if (direct && S.hist && (int)threadIdx.x < per) {   // bins above `bins`: 4 x per zero words
        const int b = 4 * threadIdx.x;
        const int c = b / per, v = F.bins + b % per;
        *reinterpret_cast<u32x4*>(S.hist + c * 256 + v) = u32x4{0, 0, 0, 0};
    }
    __syncthreads();
    if (threadIdx.x < 4 && S.sum) {
        if (direct)
            S.sum[threadIdx.x] = csum[threadIdx.x];
        else if (csum[threadIdx.x])
            atomicAdd((unsigned long long*)&S.sum[threadIdx.x], csum[threadIdx.x]);
    }
}

// Clears the histogram and sums of every segment (one work-group each).
__global__ void hist_zero_kernel(const HistFinArgs F) {
    if (F.guard && *F.guard == 0) return;
    const HistSeg& S = F.segs ? F.segs[blockIdx.x] : F.one;
    for (int b = threadIdx.x; b < 1024; b += blockDim.x)
        if (S.hist) S.hist[b] = 0;
    if (threadIdx.x < 4 && S.sum) S.sum[threadIdx.x] = 0;
}

__global__ void while_init_kernel(uint32_t* st) {
    if (threadIdx.x == 0) {
        st[0] = 1u;
        st[1] = 0u;
    }
}

// One work-group of kStepThreads threads.  Every thread reads the flag before
// thread 0 may clear it, so a finished loop merges nothing and a running one
// merges the whole histogram.
constexpr int kStepThreads = 256;
__global__ void __launch_bounds__(kStepThreads) while_step_kernel(uint32_t* st, const uint64_t* sum,
                                                                 const WhileCond c, const WhileMerge M,
                                                                 uint32_t* count_out) {
    const uint32_t running = st[0];
    __syncthreads();
    if (running == 0u) return;
    if (M.acc_hist)
        for (int b = threadIdx.x; b < 1024; b += kStepThreads) M.acc_hist[b] += M.it_hist[b];
    if (M.acc_sum && threadIdx.x < 4) M.acc_sum[threadIdx.x] += M.it_sum[threadIdx.x];
    if (threadIdx.x != 0) return;
    const uint32_t n = st[1] + 1u;
    st[1] = n;
    *count_out = n;
    uint64_t* prev = reinterpret_cast<uint64_t*>(st + 2);
    const uint64_t s = sum[c.channel];
    bool go = true;
    uint64_t v = s;
    if (c.kind == 1) {
        v = s >= *prev ? s - *prev : *prev - s;
        *prev = s;
    }
    if (c.kind == 0 || n > 1u) {
        switch (c.cmp) {
            case 0: go = v > c.threshold; break;
            case 1: go = v >= c.threshold; break;
            case 2: go = v < c.threshold; break;
            default: go = v <= c.threshold; break;
        }
    }
    if (!go || n >= (uint32_t)c.max) st[0] = 0u;
}

// Copies src to dst (nvec 16-byte vectors, then 4-byte words up to `words`)
// when max - (iterations run) is odd: the last iteration then wrote src.
__global__ void while_copy_kernel(const uint32_t* st, const uint32_t* src, uint32_t* dst, uint64_t words,
                                  uint64_t nvec, uint32_t max) {
    if ((max - st[1]) % 2u == 0u) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
        reinterpret_cast<u32x4*>(dst)[i] = reinterpret_cast<const u32x4*>(src)[i];
    for (uint64_t i = nvec * 4 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        dst[i] = src[i];
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------------------ host side
static_assert(kHistWgChan == kHistWgWords, "histogram layout");

int hist_copies_log2(int bins, int words) {
    int ks = 0;
    while ((bins << (ks + 1)) <= words) ++ks;
    return ks;
}

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
    int fl;   // compile-time mirror flags, -1 = from the arguments
    img_kfn fn;
    batch_kfn bfn;
    const char* name;
};

#define SKEL_IMG_ENTRY(P, Q, B, Hh, FL, NAME) \
    {P, Q, B, Hh, FL, img_band_kernel<P, Q, B, Hh, FL>, img_batch_kernel<P, Q, B, Hh, FL>, NAME}
// Without a stencil the input is never mirrored (mirrors fold into the
// output address), so those chains need FL 0 and 2 only.
#define SKEL_IMG_POINT(P, Hh, NAME) SKEL_IMG_ENTRY(P, 0, false, Hh, 0, NAME), SKEL_IMG_ENTRY(P, 0, false, Hh, 2, NAME)
#define SKEL_IMG_STENCIL(P, Hh, NAME)                                           \
    SKEL_IMG_ENTRY(P, 0, true, Hh, 0, NAME), SKEL_IMG_ENTRY(P, 0, true, Hh, 2, NAME), \
        SKEL_IMG_ENTRY(P, 0, true, Hh, -1, NAME)

// Specialised chains: 1 = noise, 2 = solarise, 9 = noise then solarise.
static const ImgEntry kImgTable[] = {
    SKEL_IMG_POINT(0, false, "img_copy"),
    SKEL_IMG_POINT(1, false, "img_noise"),
    SKEL_IMG_POINT(2, false, "img_solarise"),
    SKEL_IMG_POINT(0, true, "img_reduce"),
    SKEL_IMG_POINT(9, false, "img_noise_sol"),
    SKEL_IMG_POINT(9, true, "img_noise_sol_reduce"),
    SKEL_IMG_STENCIL(0, false, "img_blur"),
    SKEL_IMG_STENCIL(0, true, "img_blur_reduce"),
    SKEL_IMG_STENCIL(9, false, "img_noise_sol_blur"),
    SKEL_IMG_STENCIL(9, true, "img_noise_sol_blur_reduce"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, false, false, -1, "img_generic"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, false, true, -1, "img_generic_reduce"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, true, false, -1, "img_generic_blur"),
    SKEL_IMG_ENTRY(kGeneric, kGeneric, true, true, -1, "img_generic_blur_reduce"),
};

static const ImgEntry* find_entry(const OpList& pre, const OpList& post, bool blur, bool hist, int in_flip,
                                  int out_flip, int variant) {
    const int pe = encode_ops(pre), qe = encode_ops(post);
    const int fl = (in_flip ? 1 : 0) | (out_flip ? 2 : 0);
    const int n = (int)(sizeof(kImgTable) / sizeof(kImgTable[0]));
    if (variant == 0 && pre.n <= 6 && post.n <= 6) {
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < n; ++i) {
                const ImgEntry& e = kImgTable[i];
                if (e.pre == pe && e.post == qe && e.blur == blur && e.hist == hist && e.fl == (pass ? -1 : fl))
                    return &e;
            }
    }
    for (int i = 0; i < n; ++i) {
        const ImgEntry& e = kImgTable[i];
        if (e.pre == kGeneric && e.blur == blur && e.hist == hist) return &e;
    }
    return nullptr;
}

int img_waves_per_cu(const ImgGroupArgs& a, bool blur, bool hist, int wg, int variant) {
    const ImgEntry* e = find_entry(a.pre, a.post, blur, hist, a.in_flip, a.out_flip, variant);
    int nb = 0;
    if (!e || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(e->fn), wg, 0) !=
                  hipSuccess ||
        nb <= 0) {
        (void)hipGetLastError();
        return 16;
    }
    return nb * (wg / 64);
}

const char* img_kernel_name(const ImgGroupArgs& a, bool blur, bool hist, int variant) {
    const ImgEntry* e = find_entry(a.pre, a.post, blur, hist, a.in_flip, a.out_flip, variant);
    return e ? e->name : "";
}

hipError_t launch_img_group(const ImgGroupArgs& a, bool blur, bool hist, int wg, int variant, hipStream_t s,
                            const char** kname, hipEvent_t t0, hipEvent_t t1) {
    const ImgEntry* e = find_entry(a.pre, a.post, blur, hist, a.in_flip, a.out_flip, variant);
    if (!e) return hipErrorInvalidValue;
    if (kname) *kname = e->name;
    if (a.ntiles <= 0) {
        // nothing to launch: the requested events still mark this point
        hipError_t r = t0 ? hipEventRecord(t0, s) : hipSuccess;
        if (r == hipSuccess && t1) r = hipEventRecord(t1, s);
        return r;
    }
    const int waves = wg / 64;
    const int grid = (a.ntiles + waves - 1) / waves;
    if (t0 || t1) {
        // the events take their timestamps from the kernel's own dispatch,
        // so they bracket its execution and nothing else
        ImgGroupArgs arg = a;
        void* args[] = {&arg};
        return hipExtLaunchKernel(reinterpret_cast<const void*>(e->fn), dim3(grid), dim3(wg), args, 0, s, t0, t1,
                                  0);
    }
    hipLaunchKernelGGL(e->fn, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_img_batch(const BatchArgs& a, int grid, int wg, hipStream_t s, const char** kname) {
    const ImgEntry* e = find_entry(a.pre, a.post, a.has_blur != 0, a.has_hist != 0, a.in_flip, a.out_flip, 0);
    if (!e) return hipErrorInvalidValue;
    if (kname) *kname = e->name;
    if (wg != 256 && wg != 128 && wg != 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(e->bfn, dim3(grid), dim3(wg), 0, s, a);
    return hipGetLastError();
}

int hist_chunk_rows(int bins) { return kSumUnroll * (kFinThreads / bins); }

hipError_t launch_hist_merge(const HistFinArgs& a, hipStream_t s) {
    if (a.bins != 128 && a.bins != 256) return hipErrorInvalidValue;
    if (a.nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(hist_merge_kernel, dim3(a.nchunks), dim3(kFinThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_hist_zero(const HistFinArgs& a, hipStream_t s) {
    if (a.nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(hist_zero_kernel, dim3(a.nseg), dim3(256), 0, s, a);
    return hipGetLastError();
}

int img_batch_blocks_per_cu(const BatchArgs& a, int wg) {
    const ImgEntry* e = find_entry(a.pre, a.post, a.has_blur != 0, a.has_hist != 0, a.in_flip, a.out_flip, 0);
    if (!e) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(e->bfn), wg, 0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_while_init(uint32_t* state, hipStream_t s) {
    hipLaunchKernelGGL(while_init_kernel, dim3(1), dim3(64), 0, s, state);
    return hipGetLastError();
}

hipError_t launch_while_step(uint32_t* state, const uint64_t* sum, const WhileCond& c, const WhileMerge& m,
                             uint32_t* count_out, hipStream_t s) {
    if (c.channel < 0 || c.channel > 3 || c.kind < 0 || c.kind > 1) return hipErrorInvalidValue;
    if (!m.acc_hist != !m.it_hist || !m.acc_sum != !m.it_sum) return hipErrorInvalidValue;
    hipLaunchKernelGGL(while_step_kernel, dim3(1), dim3(kStepThreads), 0, s, state, sum, c, m, count_out);
    return hipGetLastError();
}

hipError_t launch_while_copy(const uint32_t* state, const void* src, void* dst, uint64_t bytes, uint32_t max,
                             hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    const uint64_t words = bytes / 4;
    const bool aligned = (((uintptr_t)src | (uintptr_t)dst) & 15u) == 0;
    const uint64_t nvec = aligned ? words / 4 : 0;
    uint64_t blocks = ((aligned ? nvec : words) + 255) / 256;
    blocks = std::max<uint64_t>(1, std::min<uint64_t>(blocks, 8192));
    hipLaunchKernelGGL(while_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, state, (const uint32_t*)src,
                       (uint32_t*)dst, words, nvec, max);
    return hipGetLastError();
}

hipError_t launch_fill_u32(void* p, uint64_t nwords, uint32_t value, hipStream_t s) {
    if (nwords == 0) return hipSuccess;
    uint64_t blocks = (nwords + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, nwords, value);
    return hipGetLastError();
}

}  // namespace skel
