// Per-row dot products shared by the single-call GEMV kernels and the
// batched kernel, so both run exactly the same arithmetic on a row.
//
// A group of G lanes (G a power of two, 4..64) owns a row segment of klen
// elements; x for the segment sits in LDS.  Each lane streams 16-byte
// vectors at lane stride, U of them in flight, and returns its partial sum;
// the caller reduces the group.  The order of a lane's additions depends
// only on (G, element width, row alignment), not on U.
#pragma once

#include <type_traits>

#include "sb_device.hpp"

namespace sb {

// Plain binary64 / binary32 row segment.  ALIGNED: the row start is 16-byte
// aligned (true for every row when A and ld*sizeof(T) are), so x can be read
// from LDS as vectors; otherwise up to W-1 leading elements are peeled.
// BATCH_TAIL: the vectors left after the full batches of U (fewer than U
// per lane) are loaded as one predicated batch, all in flight together;
// otherwise one at a time (fewer registers).  SHIFTED (rows not aligned):
// LDS holds W copies of x, copy h shifted left by h elements and xstride
// elements apart, so that the x of a row peeled by h elements is read from
// copy h as aligned vectors.  EDGE_NT: the peeled elements at either end
// of an unaligned row are read with the non-temporal hint too, so that
// they allocate no cache lines (a cached read of them misses to HBM when
// other data has filled the caches since the last call: binary32 65537 x
// 4093 GEMV-N after a 2 GiB write 189 -> 175 us; with A's row ends still
// cached from the previous call the hint costs 2-3 us).  PAIRS (binary32
// rows not aligned): LDS holds 2 copies of x, copy h shifted left by h
// elements and xstride apart, and a row peeled by h elements reads its x
// from copy h % 2 as aligned 8-byte pairs.  The additions happen in the
// same order in every case.
template <typename T, int G, int U, bool ALIGNED, bool NTL, bool BATCH_TAIL = true, bool SHIFTED = false,
          bool EDGE_NT = false, bool PAIRS = false>
__device__ __forceinline__ T row_dot(const T* Ar, int64_t klen, const T* xs, int l, int64_t xstride = 0)
{
    typedef typename Vec<T>::type V;
    constexpr int W = Vec<T>::W;
    int64_t head = 0;
    if (!ALIGNED) {
        head = ((16 - (reinterpret_cast<uintptr_t>(Ar) & 15)) & 15) / sizeof(T);
        head = min(head, klen);
    }
    V acc = (V)0;
    if (!ALIGNED && l < head) acc[0] = ld_stream<NTL && EDGE_NT>(Ar + l) * xs[l];

    const int64_t nv = (klen - head) / W;
    const V* Av = reinterpret_cast<const V*>(Ar + head);
    static_assert(!PAIRS || (std::is_same<T, float>::value && !SHIFTED), "pairs: binary32, one copy mode");
    const T* xb = SHIFTED ? xs + head * xstride : PAIRS ? xs + (head & 1) * xstride + (head & ~(int64_t)1) : xs + head;
    int64_t v = l;
    // Full batches: with BATCH_TAIL as many as every lane of the group has
    // (the same count for the whole wave), the rest in one predicated batch.
    const int64_t vfull = BATCH_TAIL ? nv / (U * G) * (U * G) : nv - (U - 1) * G;
    for (; v < vfull && v + (U - 1) * G < nv; v += U * G) {
        V av[U];
#pragma unroll
        for (int u = 0; u < U; ++u) av[u] = ld_stream<NTL>(Av + v + u * G);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = (v + u * G) * W;
            if (ALIGNED || SHIFTED) {
                acc += av[u] * *reinterpret_cast<const V*>(xb + e);
            } else if constexpr (PAIRS) {
                const v2f xa = *reinterpret_cast<const v2f*>(xb + e);
                const v2f xc = *reinterpret_cast<const v2f*>(xb + e + 2);
                acc[0] += av[u][0] * xa[0];
                acc[1] += av[u][1] * xa[1];
                acc[2] += av[u][2] * xc[0];
                acc[3] += av[u][3] * xc[1];
            } else {
#pragma unroll
                for (int q = 0; q < W; ++q) acc[q] += av[u][q] * xb[e + q];
            }
        }
    }
    if (BATCH_TAIL && v < nv) {
        // fewer than U vectors remain for this lane: one predicated batch
        // (all its loads in flight together), added in the same order
        V av[U];
#pragma unroll
        for (int u = 0; u < U; ++u) av[u] = v + u * G < nv ? ld_stream<NTL>(Av + v + u * G) : (V)0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v + u * G < nv) {
                const int64_t e = (v + u * G) * W;
#pragma unroll
                for (int q = 0; q < W; ++q) acc[q] += av[u][q] * xb[e + q];
            }
        }
        v += U * G;
    }
    for (; v < nv; v += G) {  // not taken after a batched tail
        const V av = ld_stream<NTL>(Av + v);
        const int64_t e = v * W;
#pragma unroll
        for (int q = 0; q < W; ++q) acc[q] += av[q] * xb[e + q];
    }
    const int64_t t0 = head + nv * W;  // fewer than W elements remain
    if (l < klen - t0) acc[1 % W] += ld_stream<NTL && EDGE_NT>(Ar + t0 + l) * xs[t0 + l];

    T t = acc[0];
#pragma unroll
    for (int q = 1; q < W; ++q) t += acc[q];
    return t;
}

// ---- narrow storage: bfloat16 / OCP E4M3FN codes, binary32 arithmetic ----

template <bool BF16> struct Codes;
template <> struct Codes<true> {
    typedef uint16_t code_t;
    static constexpr int PER16 = 8;  // values per 16-byte load
    __device__ static float one(uint16_t c) { return __uint_as_float((uint32_t)c << 16); }
    // 4 dwords -> 8 values, element order preserved
    __device__ static void unpack(const v4u& w, float* f)
    {
        const uint32_t d[4] = {w[0], w[1], w[2], w[3]};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            f[2 * k] = __uint_as_float(d[k] << 16);
            f[2 * k + 1] = __uint_as_float(d[k] & 0xFFFF0000u);
        }
    }
};
template <> struct Codes<false> {
    typedef uint8_t code_t;
    static constexpr int PER16 = 16;
    __device__ static float one(uint8_t c)
    {
        return __builtin_amdgcn_cvt_f32_fp8((int)c, 0);
    }
    __device__ static void unpack(const v4u& w, float* f)
    {
        const uint32_t d[4] = {w[0], w[1], w[2], w[3]};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)d[k], false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)d[k], true);
            f[4 * k] = lo[0];
            f[4 * k + 1] = lo[1];
            f[4 * k + 2] = hi[0];
            f[4 * k + 3] = hi[1];
        }
    }
};

// Partial dot products of R consecutive rows (Q0 is the first, rows ldq
// codes apart) with the staged x, for lane l of a group of G lanes.  All R
// rows must share the same 16-byte alignment.  A lane's additions happen in
// the same order for any U and R, so the result does not depend on them.
// EDGE_NT as for row_dot: the codes peeled at the row ends read with the
// non-temporal hint.  XC > 1: LDS holds XC copies of x, copy h shifted left
// by h elements and xstride elements apart, and a row peeled by h codes
// reads the x of its vectors from copy h % XC as aligned XC-element vectors
// (4: 16 bytes, 2: 8 bytes).  With one copy (XC = 1) rows with h % 4 != 0
// read x one element at a time, lanes P elements apart: a bank conflict of
// every lane pair 32/P apart.
template <class C, int G, int U, int R, bool NTL, bool BATCH_TAIL = true, bool EDGE_NT = false, int XC = 1>
__device__ __forceinline__ void tile_dot(const typename C::code_t* Q0, int64_t ldq, int64_t klen,
                                         const float* xs, int l, float (&t)[R], int64_t xstride = 0)
{
    typedef typename C::code_t code_t;
    constexpr int P = C::PER16;
    int64_t head = ((16 - (reinterpret_cast<uintptr_t>(Q0) & 15)) & 15) / sizeof(code_t);
    head = min(head, klen);
    float acc[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0f;
    for (int64_t e = l; e < head; e += G) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][0] += C::one(ld_stream<NTL && EDGE_NT>(Q0 + r * ldq + e)) * xs[e];
    }
    const int64_t nv = (klen - head) / P;
    static_assert(XC == 1 || XC == 2 || XC == 4, "x copies");
    const int64_t hs = XC > 1 ? (head & (XC - 1)) : 0;
    const float* xb = xs + hs * xstride + head - hs;
    const bool xal = XC > 1 || ((head * 4) & 15) == 0;
    const v4u* Qv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) Qv[r] = reinterpret_cast<const v4u*>(Q0 + r * ldq + head);
    int64_t v = l;
    // Full batches: with BATCH_TAIL as many as every lane of the group has
    // (the same count for the whole wave), the rest in one predicated batch.
    const int64_t vfull = BATCH_TAIL ? nv / (U * G) * (U * G) : nv - (U - 1) * G;
    // Main loop: U loads per row in flight, then one straight-line step per
    // load (the x-alignment choice is hoisted so each step is one block).
    auto main_loop = [&](auto xal_tag) {
        constexpr bool XAL = decltype(xal_tag)::value;
        for (; v < vfull && v + (U - 1) * G < nv; v += U * G) {
            v4u wv[U][R];
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int r = 0; r < R; ++r) wv[u][r] = ld_stream<NTL>(Qv[r] + v + u * G);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float* xe = xb + (v + u * G) * P;
                float xr[P];
#pragma unroll
                for (int q = 0; q < P; q += 4) {
                    if constexpr (XAL && XC == 2) {
                        const v2f xa = *reinterpret_cast<const v2f*>(xe + q);
                        const v2f xc = *reinterpret_cast<const v2f*>(xe + q + 2);
                        xr[q] = xa[0];
                        xr[q + 1] = xa[1];
                        xr[q + 2] = xc[0];
                        xr[q + 3] = xc[1];
                    } else if constexpr (XAL) {
                        const v4f xv = *reinterpret_cast<const v4f*>(xe + q);
                        xr[q] = xv[0];
                        xr[q + 1] = xv[1];
                        xr[q + 2] = xv[2];
                        xr[q + 3] = xv[3];
                    } else {
                        xr[q] = xe[q];
                        xr[q + 1] = xe[q + 1];
                        xr[q + 2] = xe[q + 2];
                        xr[q + 3] = xe[q + 3];
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float f[P];
                    C::unpack(wv[u][r], f);
#pragma unroll
                    for (int q = 0; q < P; ++q) acc[r][q & 3] += f[q] * xr[q];
                }
                // Keep each step's LDS reads and decodes inside the step:
                // hoisted all together they need more than 200 VGPRs.  The
                // global loads above are already in flight.
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    if (xal) main_loop(std::true_type{});
    else main_loop(std::false_type{});
    if (BATCH_TAIL && v < nv) {
        // fewer than U vectors remain for this lane: one predicated batch
        v4u wv[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int r = 0; r < R; ++r) wv[u][r] = v + u * G < nv ? ld_stream<NTL>(Qv[r] + v + u * G) : v4u{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v + u * G < nv) {
                const float* xe = xb + (v + u * G) * P;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float f[P];
                    C::unpack(wv[u][r], f);
#pragma unroll
                    for (int q = 0; q < P; ++q) acc[r][q & 3] += f[q] * xe[q];
                }
            }
        }
        v += U * G;
    }
    for (; v < nv; v += G) {  // not taken after a batched tail
        const float* xe = xb + v * P;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float f[P];
            C::unpack(ld_stream<NTL>(Qv[r] + v), f);
#pragma unroll
            for (int q = 0; q < P; ++q) acc[r][q & 3] += f[q] * xe[q];
        }
    }
    for (int64_t e = head + nv * P + l; e < klen; e += G) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][1] += C::one(ld_stream<NTL && EDGE_NT>(Q0 + r * ldq + e)) * xs[e];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]);
}

// x transposed by residue, for rows that are not 16-byte aligned: element e
// of the staged segment sits at xt[(e % P) * NP + e / P], NP >= klen / P
// rounded up (odd, so that staging writes spread over the banks).
// A row peeled by h codes pairs code q of its vector v with element
// h + v P + q, whose slot is off_q + v with off_q fixed for the row, so the
// lanes of a group (consecutive v) read consecutive dwords whatever h is.
// In the plain layout those lanes read dwords P apart, a bank conflict of
// every lane pair 32/P apart (E4M3 rows of 16383 codes: 1.2 TB/s, bound by
// the LDS).
template <int P>
__device__ __forceinline__ int64_t xt_slot(int64_t e, int64_t NP)
{
    return (e & (P - 1)) * NP + (e >> __builtin_ctz(P));
}

// One row's partial dot product against the transposed x: the same loads
// and the same additions in the same order as tile_dot with R = 1.
template <class C, int G, int U, bool NTL, bool BATCH_TAIL = true, bool EDGE_NT = false>
__device__ __forceinline__ float tile_dot_xt(const typename C::code_t* Q0, int64_t klen, const float* xt, int64_t NP,
                                             int l)
{
    constexpr int P = C::PER16;
    typedef typename C::code_t code_t;
    int64_t head = ((16 - (reinterpret_cast<uintptr_t>(Q0) & 15)) & 15) / sizeof(code_t);
    head = min(head, klen);
    // one row per wave: the slot offsets below are wave-uniform (scalar)
    if constexpr (G == 64) head = __builtin_amdgcn_readfirstlane((int32_t)head);
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t e = l; e < head; e += G) acc[0] += C::one(ld_stream<NTL && EDGE_NT>(Q0 + e)) * xt[xt_slot<P>(e, NP)];
    const int64_t nv = (klen - head) / P;
    const v4u* Qv = reinterpret_cast<const v4u*>(Q0 + head);
    // slot of element head + v P + q: off[q] + v (head < P, so at most one carry)
    int32_t off[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int32_t hq = (int32_t)head + q;
        off[q] = (hq & (P - 1)) * (int32_t)NP + (hq >= P ? 1 : 0);
    }
    auto step = [&](const v4u& wv, int64_t v) {
        float f[P];
        C::unpack(wv, f);
        const float* xv = xt + v;
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q & 3] += f[q] * xv[off[q]];
    };
    int64_t v = l;
    const int64_t vfull = BATCH_TAIL ? nv / (U * G) * (U * G) : nv - (U - 1) * G;
    for (; v < vfull && v + (U - 1) * G < nv; v += U * G) {
        v4u wv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) wv[u] = ld_stream<NTL>(Qv + v + u * G);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            step(wv[u], v + u * G);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (BATCH_TAIL && v < nv) {
        v4u wv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) wv[u] = v + u * G < nv ? ld_stream<NTL>(Qv + v + u * G) : v4u{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v + u * G < nv) step(wv[u], v + u * G);
        v += U * G;
    }
    for (; v < nv; v += G) step(ld_stream<NTL>(Qv + v), v);  // not taken after a batched tail
    for (int64_t e = head + nv * P + l; e < klen; e += G)
        acc[1] += C::one(ld_stream<NTL && EDGE_NT>(Q0 + e)) * xt[xt_slot<P>(e, NP)];
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

}  // namespace sb
