// Arithmetic in F_p for 31-bit primes on gfx950.
//
// Residues are uint32 in [0, p) with 2 <= p < 2^31.  The paper gets fast
// reduction by making p a compile-time constant (Sec. 3.2, "Meta-programming";
// Sec. 3.4).  Here p is a run-time value (a batch may hold one prime per
// system), so the constants each method needs are computed once per prime on
// the host (FieldConst) and the hot loop uses
//   - Shoup's multiplication by a fixed operand with a precomputed quotient
//     (V. Shoup, NTL; D. Harvey, "Faster arithmetic for number-theoretic
//     transforms", 2014): w' = floor(w * 2^32 / p), then for any a < 2^32
//     q = hi32(a * w'), r = a*w - q*p (mod 2^32) lies in [0, 2p);
//   - for p = 2^31 - 1 the Mersenne fold z mod p = (z & p) + (z >> 31);
//   - for a product of two run-time residues, an FP64 reduction: with
//     h = fl(a*b) and l = a*b - h (exact by FMA), q = floor(h / p) is within
//     one of the true quotient, and a*b - q*p = fma(-q, p, h) + l is computed
//     exactly, then corrected into [0, p).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace linac {

static constexpr uint32_t kMersenne31 = 0x7fffffffu;

struct FieldConst {
    uint32_t p;
    uint32_t pprime;  // -p^-1 mod 2^32 (Montgomery; p odd)
    uint32_t r2;      // 2^64 mod p
    uint32_t pad;
    double dp;        // (double)p
    double pinv;      // fl(1 / p)
    double two32_p;   // fl(2^32 / p)
};

__host__ inline FieldConst make_field(uint32_t p) {
    FieldConst f;
    f.p = p;
    // p^-1 mod 2^32 by Newton's iteration x <- x (2 - p x), exact bits doubling
    uint32_t x = p;
    for (int i = 0; i < 5; ++i) x *= 2u - p * x;
    f.pprime = (uint32_t)(0u - x);
    const uint64_t r1 = (uint64_t)(((uint64_t)1 << 32) % p);
    f.r2 = (uint32_t)(r1 * r1 % p);
    f.pad = 0;
    f.dp = (double)p;
    f.pinv = 1.0 / (double)p;
    f.two32_p = 4294967296.0 / (double)p;
    return f;
}

__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t p) {
    uint32_t s = a + b;  // < 2^32 since a, b < 2^31
    uint32_t t = s - p;
    return t < s ? t : s;  // s >= p  <=>  no wrap in s - p
}

// (x - t) mod p for x, t in [0, p).  If x >= t the difference is the answer;
// otherwise it wrapped to >= 2^32 - p > p and adding p gives the answer.
__device__ __forceinline__ uint32_t sub_mod(uint32_t x, uint32_t t, uint32_t p) {
    uint32_t d = x - t;
    uint32_t e = d + p;
    return d < e ? d : e;
}

// Reduce r in [0, 2p) to [0, p).
__device__ __forceinline__ uint32_t reduce_2p(uint32_t r, uint32_t p) {
    uint32_t t = r - p;
    return t < r ? t : r;
}

// a * b mod p for run-time residues a, b (FP64, exact; see header comment).
__device__ __forceinline__ uint32_t mul_mod(uint32_t a, uint32_t b, const FieldConst& F) {
    double da = (double)a, db = (double)b;
    double h = da * db;
    double l = __fma_rn(da, db, -h);
    double q = floor(h * F.pinv);
    double r = __fma_rn(-q, F.dp, h) + l;  // exact: a*b - q*p in [-p, 2p)
    if (r < 0.0) r += F.dp;
    if (r >= F.dp) r -= F.dp;
    return (uint32_t)r;
}

// Shoup quotient w' = floor(w * 2^32 / p) for a fixed multiplier w < p.
__device__ __forceinline__ uint32_t shoup_quot(uint32_t w, const FieldConst& F) {
    double est = floor((double)w * F.two32_p);  // within one of the true value
    uint32_t q = (uint32_t)est;
    // remainder w*2^32 - q*p as a signed 64-bit value, then step q by one
    int64_t rem = (int64_t)(((uint64_t)w << 32) - (uint64_t)q * (uint64_t)F.p);
    if (rem < 0) q -= 1;
    else if (rem >= (int64_t)F.p) q += 1;
    return q;
}

// a * w mod p in [0, 2p) with the Shoup quotient wq of w.
__device__ __forceinline__ uint32_t shoup_mul_lazy(uint32_t a, uint32_t w, uint32_t wq, uint32_t p) {
    uint32_t q = __umulhi(a, wq);
    return a * w - q * p;
}

// z mod (2^31 - 1) for z < 2^62.
__device__ __forceinline__ uint32_t mersenne_reduce(uint64_t z) {
    uint32_t lo = (uint32_t)z & kMersenne31;
    uint32_t hi = (uint32_t)(z >> 31);
    uint32_t s = lo + hi;  // < 2^32
    return reduce_2p(s, kMersenne31);
}

// Montgomery reduction (P. Montgomery, "Modular multiplication without trial
// division", 1985) with R = 2^32: for T < p * 2^32 returns T / R mod p.  For
// p < 2^31, T + m p < 2^64 and the quotient is below 2p.
__device__ __forceinline__ uint32_t redc(uint64_t T, uint32_t p, uint32_t pprime) {
    const uint32_t m = (uint32_t)T * pprime;
    const uint64_t t = (T + (uint64_t)m * p) >> 32;
    return t >= p ? (uint32_t)(t - p) : (uint32_t)t;
}

// a^-1 = a^(p-2) mod p (Fermat) by square-and-multiply in Montgomery form.  It
// uses 32-bit integer multiplies only, so for a wave-uniform argument the
// compiler keeps it on the scalar unit, off the vector pipeline and short in
// latency.  p = 2 (even, no Montgomery form) has the single unit 1.
__device__ inline uint32_t inv_mod_fermat(uint32_t a, const FieldConst& F) {
    const uint32_t p = F.p;
    if (p == 2) return a;
    const uint32_t pp = F.pprime;
    uint32_t x = redc((uint64_t)a * F.r2, p, pp);  // a R mod p
    uint32_t r = redc((uint64_t)F.r2, p, pp);      // R mod p (Montgomery form of 1)
    for (uint32_t e = p - 2; e != 0; e >>= 1) {
        if (e & 1) r = redc((uint64_t)r * x, p, pp);
        x = redc((uint64_t)x * x, p, pp);
    }
    return redc((uint64_t)r, p, pp);
}

// Modular inverse of a != 0 by the extended Euclidean algorithm.  Returns 0 for
// a = 0 (never used as a pivot).
__device__ inline uint32_t inv_mod(uint32_t a, uint32_t p) {
    int64_t t = 0, nt = 1;
    uint32_t r = p, nr = a;
    while (nr != 0) {
        uint32_t q = r / nr;
        int64_t tmp = t - (int64_t)q * nt;
        t = nt;
        nt = tmp;
        uint32_t rr = r - q * nr;
        r = nr;
        nr = rr;
    }
    if (t < 0) t += p;
    return (uint32_t)t;
}

// The balanced representative of a residue: v - p when v > (p - 1) / 2, so
// |result| <= (p - 1) / 2 (below 2^30 for p < 2^31).
__device__ __forceinline__ int32_t centre(uint32_t v, uint32_t p) {
    return v > (p - 1) / 2 ? (int32_t)v - (int32_t)p : (int32_t)v;
}

// Four signed base-256 digits of x (|x| <= 2^30), least significant first:
// x = sum_l 256^l d[l] with every d[l] in [-128, 127].
__device__ __forceinline__ void digits4(int32_t x, int8_t d[4]) {
    for (int l = 0; l < 4; ++l) {
        const int8_t lo = (int8_t)(x & 0xff);
        d[l] = lo;
        x = (x - lo) >> 8;
    }
}

}  // namespace linac
