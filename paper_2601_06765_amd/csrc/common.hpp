// Shared device/host definitions of the gfx950 F4 library: F_p arithmetic,
// packed monomials, the dense grevlex rank, wave64 helpers, error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint8_t u8;

#define F4_WAVE 64

// ------------------------------------------------------------- F_p arithmetic
// Residues are canonical, in [0, p), at every buffer boundary; p is an odd
// prime below 2^31 (word-size regime of the section "Word-size regimes and
// overflow discipline": p < 2^(w-1) with w = 32, products exact in 64 bits).
//
// Barrett reduction (section "Barrett reduction as reciprocal
// multiplication"): with s = bitlength(p) and mu = floor(2^(2s) / p), an input
// x < 2^(2s) gets the quotient estimate q = ((x >> (s-1)) * mu) >> (s+1), which
// undershoots floor(x/p) by at most 2, so r = x - q*p needs at most two
// predicated subtractions.  Both factors of the estimate fit in 32 bits, so it
// costs one 32x32->64 multiply; q*p is one more.
struct Fp {
    u32 p;   // modulus
    u32 s;   // bit length of p
    u32 mu;  // floor(2^(2s) / p)  (< 2^32 for odd p)
    u32 mu32; // floor(2^32 / p): single-word Barrett for any x < 2^32
    u32 r32;  // 2^32 mod p
    float finv;   // 1/p rounded to float (quotient estimate for p < 2^16)
};

static inline Fp make_fp(u32 p) {
    Fp f;
    f.p = p;
    f.s = 0;
    while ((1ull << f.s) <= p) ++f.s;
    unsigned __int128 num = (unsigned __int128)1 << (2 * f.s);
    f.mu = (u32)(num / p);
    f.mu32 = (u32)((1ull << 32) / p);
    f.r32 = (u32)((1ull << 32) % p);
    f.finv = 1.0f / (float)p;
    return f;
}

// x < 2^(2s)  ->  x mod p
__host__ __device__ __forceinline__ u32 fp_reduce(const Fp& f, u64 x) {
    u32 hi = (u32)(x >> (f.s - 1));
    u32 q = (u32)(((u64)hi * f.mu) >> (f.s + 1));
    u64 r = x - (u64)q * f.p;
    r = (r >= f.p) ? r - f.p : r;
    r = (r >= f.p) ? r - f.p : r;
    return (u32)r;
}

// x < 2^32  ->  x mod p   (quotient estimate off by at most one, any p < 2^31)
__host__ __device__ __forceinline__ u32 fp_reduce32(const Fp& f, u32 x) {
#ifdef __HIP_DEVICE_COMPILE__
    u32 q = __umulhi(x, f.mu32);
#else
    u32 q = (u32)(((u64)x * f.mu32) >> 32);
#endif
    u32 r = x - q * f.p;
    return (r >= f.p) ? r - f.p : r;
}

// any 64-bit x  ->  x mod p: split into 32-bit halves when x >= 2^(2s)
__host__ __device__ __forceinline__ u32 fp_reduce_any(const Fp& f, u64 x) {
    if ((x >> (2 * f.s)) == 0) return fp_reduce(f, x);
    u32 h = fp_reduce32(f, (u32)(x >> 32)), l = fp_reduce32(f, (u32)x);
    return fp_reduce(f, (u64)h * f.r32 + l);
}

// low 32 bits of the product of the low 24 bits of a and b, unsigned (the
// runtime's __umul24 returns int, which would sign-extend when widened)
__device__ __forceinline__ u32 mul24(u32 a, u32 b) { return (u32)__umul24(a, b); }

// a*b mod p for p < 2^16 and a, b < p, with full-rate 24-bit multiplies: the
// product x < 2^32 is exact in the low word; the float estimate of x/p has
// relative error below 2^-22, so with x/p < 2^16 its truncation q is off by at
// most one and x - q*p lies in [-p, 2p); two unsigned min steps (an add that
// wraps picks the corrected value) bring it to [0, p).
__device__ __forceinline__ u32 fp_mul16(const Fp& f, u32 a, u32 b) {
    const u32 x = mul24(a, b);
    const u32 q = (u32)((float)x * f.finv);
    u32 r = x - mul24(q, f.p);
    r = min(r, r + f.p);
    return min(r, r - f.p);
}

// a*b mod p for p < 2^16 and a, b < p: the product is exact in one word and
// the one-word Barrett step reduces it (six full-rate instructions on gfx950,
// where 32-bit integer multiplies issue at the full vector rate; the modular
// inner-loop microbenchmark measures it well ahead of the 24-bit form above).
__host__ __device__ __forceinline__ u32 fp_mul32(const Fp& f, u32 a, u32 b) { return fp_reduce32(f, a * b); }

// (a + b*c) mod p for canonical a, b, c: equation "mod-fma"
__host__ __device__ __forceinline__ u32 fp_fma(const Fp& f, u32 a, u32 b, u32 c) {
    return fp_reduce(f, (u64)a + (u64)b * c);
}

template <bool SMALL>
__host__ __device__ __forceinline__ u32 fp_fma_t(const Fp& f, u32 a, u32 b, u32 c) {
    if (SMALL) return fp_reduce32(f, a + b * c);  // a + b*c <= p(p-1) < 2^32
    return fp_reduce(f, (u64)a + (u64)b * c);
}

__host__ __device__ __forceinline__ u32 fp_mul(const Fp& f, u32 a, u32 b) { return fp_reduce(f, (u64)a * b); }

__host__ __device__ __forceinline__ u32 fp_neg(const Fp& f, u32 a) { return a ? f.p - a : 0; }

// a^-1 by Fermat's little theorem: a^(p-2)
__host__ __device__ inline u32 fp_inv(const Fp& f, u32 a) {
    u32 e = f.p - 2, r = 1, b = a;
    while (e) {
        if (e & 1) r = fp_mul(f, r, b);
        b = fp_mul(f, b, b);
        e >>= 1;
    }
    return r;
}

// Montgomery multiplication (section "Montgomery multiplication and domain
// reuse") with R = 2^32, pinv = -p^-1 mod 2^32: REDC(a*b) = a*b*R^-1 mod p with
// one conditional subtraction (any odd p < 2^31: t + q*p < 2^63 + 2^62 and the
// quotient by R is below 2p).  Measured against the Barrett forms by the modular
// inner-loop microbenchmark; the elimination kernels keep standard residues.
struct Mont {
    u32 p, pinv, r2;  // r2 = R^2 mod p
};
static inline Mont make_mont(u32 p) {
    Mont m;
    m.p = p;
    u32 inv = 1;  // Newton iteration for p^-1 mod 2^32
    for (int i = 0; i < 5; ++i) inv *= 2 - p * inv;
    m.pinv = (u32)(0u - inv);
    u64 r = (1ull << 32) % p;
    m.r2 = (u32)((r * r) % p);
    return m;
}
__host__ __device__ __forceinline__ u32 mont_mul(const Mont& m, u32 a, u32 b) {
    u64 t = (u64)a * b;
    u32 q = (u32)t * m.pinv;
    u64 u = (t + (u64)q * m.p) >> 32;
    return (u >= m.p) ? (u32)(u - m.p) : (u32)u;
}

// ------------------------------------------------------------------ monomials
// P word: degree in bits 56..63, exponent a_i (i = 1..n) in a lane of w bits at
// offset w*(i-1).  Section "Monomial keys": key = (deg, tie) in one word.
__host__ __device__ __forceinline__ u32 lane_bits(u32 n) {
    if (n == 0 || n > 14) return 0;
    u32 w = 56 / n;
    return w > 8 ? 8 : w;
}
__host__ __device__ __forceinline__ u32 mono_deg(u64 P) { return (u32)(P >> 56); }
__host__ __device__ __forceinline__ u32 mono_exp(u64 P, u32 i, u32 w) {  // i is 0-based
    return (u32)((P >> (w * i)) & ((1u << w) - 1));
}
// Order key: larger key = larger monomial under grevlex (x_1 > ... > x_n).
// Complementing the lanes makes a smaller exponent of x_n (top lane) win.
__host__ __device__ __forceinline__ u64 mono_order_key(u64 P, u32 n, u32 w) {
    u64 lanemask = (n * w >= 64) ? ~0ull : ((1ull << (n * w)) - 1);
    return P ^ lanemask;
}
__host__ __device__ __forceinline__ bool mono_divides(u64 a, u64 b, u32 n, u32 w) {
    if (mono_deg(a) > mono_deg(b)) return false;
    for (u32 i = 0; i < n; ++i)
        if (mono_exp(a, i, w) > mono_exp(b, i, w)) return false;
    return true;
}
__host__ __device__ __forceinline__ u64 mono_lcm(u64 a, u64 b, u32 n, u32 w) {
    u64 r = 0;
    u32 d = 0;
    for (u32 i = 0; i < n; ++i) {
        u32 x = mono_exp(a, i, w), y = mono_exp(b, i, w);
        u32 m = x > y ? x : y;
        r |= (u64)m << (w * i);
        d += m;
    }
    return r | ((u64)d << 56);
}

// Dense grevlex rank over Mon_{<=D}: rank 0 is x_1^D, ranks increase as the
// monomial decreases.  Degree-e monomials occupy [N(n,D) - N(n,e), ...), with
// N(n,e) = C(n+e, e) (equation "monomial-count").  Inside one degree, grevlex
// descending is lexicographic ascending on (a_n, a_{n-1}, ..., a_2); counting
// the smaller tuples level by level gives
//   rank_e(a) = sum_{i=2..n} [ C(R_i+i-1, i-1) - C(R_i-a_i+i-1, i-1) ],
//   R_n = e, R_{i-1} = R_i - a_i   (hockey-stick identity).
// The binomial table binom[x*(BSTRIDE)+y] = C(x, y) for x <= n+D+1, y <= n.
#define F4_BSTRIDE 16
struct RankTab {
    u32 n, w, D;
    u32 nmax;        // N(n, D)
    const u32* binom;  // device pointer, (n+D+2) x F4_BSTRIDE
};

__host__ __device__ __forceinline__ u32 binom_at(const u32* B, u32 x, u32 y) { return B[x * F4_BSTRIDE + y]; }

#define F4_BAD_RANK 0xffffffffu
// Returns F4_BAD_RANK for a word that is not a monomial of degree <= D (degree
// field above D, or lanes that do not add up to the degree field).
__host__ __device__ __forceinline__ u32 mono_rank(u64 P, u32 n, u32 w, u32 D, const u32* B) {
    u32 e = mono_deg(P);
    if (e > D) return F4_BAD_RANK;
    // base(e) = N(n, D) - N(n, e) = C(n+D, n) - C(n+e, n)
    u32 rank = binom_at(B, n + D, n) - binom_at(B, n + e, n);
    u32 R = e;
    for (u32 i = n; i >= 2; --i) {
        u32 a = mono_exp(P, i - 1, w);
        if (a > R) return F4_BAD_RANK;
        rank += binom_at(B, R + i - 1, i - 1) - binom_at(B, R - a + i - 1, i - 1);
        R -= a;
    }
    if (mono_exp(P, 0, w) != R) return F4_BAD_RANK;
    return rank;
}

__host__ __device__ inline u64 mono_unrank(u32 q, u32 n, u32 w, u32 D, const u32* B) {
    // find the degree block
    u32 e = D;
    u32 base = 0;
    for (;;) {
        u32 cnt = binom_at(B, n + e - 1, n - 1);  // monomials of degree exactly e
        if (q < base + cnt || e == 0) break;
        base += cnt;
        --e;
    }
    u32 qq = q - base, R = e;
    u64 P = (u64)e << 56;
    for (u32 i = n; i >= 2; --i) {
        u32 top = binom_at(B, R + i - 1, i - 1);
        u32 a = 0;
        while (a < R && top - binom_at(B, R - (a + 1) + i - 1, i - 1) <= qq) ++a;
        qq -= top - binom_at(B, R - a + i - 1, i - 1);
        P |= (u64)a << (w * (i - 1));
        R -= a;
    }
    P |= (u64)R;  // a_1
    return P;
}

// --------------------------------------------------------------- wave helpers
__device__ __forceinline__ u64 wave_ballot(bool pred) { return __ballot(pred); }
__device__ __forceinline__ u32 lane_id() { return threadIdx.x & (F4_WAVE - 1); }

// Exclusive scan of one value per thread across the workgroup (blockDim a
// multiple of 64, at most 1024): wave scans with shuffles, then a scan of the
// wave totals by the first wave.  s_wave needs 33 words.  *total = block sum.
__device__ __forceinline__ u32 block_exclusive_scan(u32 v, u32* s_wave, u32* total) {
    const u32 lane = lane_id(), wave = threadIdx.x / F4_WAVE;
    u32 x = v;
#pragma unroll
    for (u32 d = 1; d < F4_WAVE; d <<= 1) {
        u32 y = __shfl_up(x, d, F4_WAVE);
        if (lane >= d) x += y;
    }
    if (lane == F4_WAVE - 1) s_wave[wave] = x;
    __syncthreads();
    const u32 nw = blockDim.x / F4_WAVE;
    if (wave == 0) {
        u32 t = lane < nw ? s_wave[lane] : 0;
        u32 z = t;
#pragma unroll
        for (u32 d = 1; d < F4_WAVE; d <<= 1) {
            u32 y = __shfl_up(z, d, F4_WAVE);
            if (lane >= d) z += y;
        }
        if (lane < nw) s_wave[lane] = z - t;
        if (lane == nw - 1) s_wave[32] = z;
    }
    __syncthreads();
    u32 r = s_wave[wave] + x - v;
    *total = s_wave[32];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------- errors
struct F4Error {
    int code;
    std::string msg;
};

#define F4_HIP_TRY(expr)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            throw F4Error{e_ == hipErrorOutOfMemory ? 3 : 5,                                     \
                          std::string(#expr) + ": " + hipGetErrorString(e_)};                   \
    } while (0)

#define F4_LAUNCH_CHECK() F4_HIP_TRY(hipGetLastError())

static inline u32 ceil_div(u64 a, u64 b) { return (u32)((a + b - 1) / b); }
