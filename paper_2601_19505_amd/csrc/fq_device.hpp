// fq_device.hpp -- device building blocks of the FCIQMC step for gfx950.
//
//  * Philox4x32-10 counter-based draws (Salmon et al., SC'11), keyed on
//    (seed, step, address, attempt) so that the spawn set does not depend on
//    the thread schedule.
//  * Exact order-independent accumulation: every contribution is converted to
//    a signed 128-bit fixed-point integer with 80 fractional bits and summed
//    with integer adds (LDS or global atomics); the total is rounded once to
//    the nearest double.  For |contribution| >= 2^-28 and |sum| < 2^46 this
//    is the exactly rounded sum, identical for every order of summation;
//    a contribution that is not a multiple of 2^-80 is reported (inexact).
//  * Bit operations on the unary Fock address of Sec. 6.1 (N+M-1 bits, mode 1
//    in the low bits) held in one or two 64-bit words.
//  * The two Hamiltonians: the real-space ring of Sec. 2 (Eq.
//    bose-hubbard-hamiltonian) and the momentum-space model of Sec. 6.3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fq {

typedef unsigned long long u64;
typedef long long i64;
typedef uint32_t u32;

// ---------------------------------------------------------------- global memory

// The descriptors hold generic pointers.  Hot accesses of device memory go
// through these views, so that they compile to global (not flat) memory
// instructions: flat loads also count against the LDS wait counter, so every
// wait for an LDS result would drain the HBM loads in flight as well.
#if defined(__HIP_DEVICE_COMPILE__)
#define FQ_GAS __attribute__((address_space(1)))
#else
#define FQ_GAS  // the host pass only parses device functions
#endif
template <class T> __device__ __forceinline__ const FQ_GAS T *gmem(const T *p) { return (const FQ_GAS T *)p; }
template <class T> __device__ __forceinline__ FQ_GAS T *gmem(T *p) { return (FQ_GAS T *)p; }
// device-scope relaxed add (the ordering of atomicAdd) on device memory
__device__ __forceinline__ int gatomic_add(int *p, int v)
{
    return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- bits

__device__ __forceinline__ u64 dbits(double d) { return (u64)__double_as_longlong(d); }
__device__ __forceinline__ double bitsd(u64 b) { return __longlong_as_double((long long)b); }

struct U128 {
    u64 lo, hi;
};

__device__ __forceinline__ U128 operator&(U128 a, U128 b) { return {a.lo & b.lo, a.hi & b.hi}; }
__device__ __forceinline__ U128 operator|(U128 a, U128 b) { return {a.lo | b.lo, a.hi | b.hi}; }
__device__ __forceinline__ U128 operator^(U128 a, U128 b) { return {a.lo ^ b.lo, a.hi ^ b.hi}; }
__device__ __forceinline__ U128 operator~(U128 a) { return {~a.lo, ~a.hi}; }
__device__ __forceinline__ bool operator==(U128 a, U128 b) { return a.lo == b.lo && a.hi == b.hi; }
__device__ __forceinline__ bool operator!=(U128 a, U128 b) { return !(a == b); }

__device__ __forceinline__ u32 shl(u32 x, int s) { return s >= 32 ? 0u : x << s; }
__device__ __forceinline__ u32 shr(u32 x, int s) { return s >= 32 ? 0u : x >> s; }
__device__ __forceinline__ u64 shl(u64 x, int s) { return s >= 64 ? 0ull : x << s; }
__device__ __forceinline__ u64 shr(u64 x, int s) { return s >= 64 ? 0ull : x >> s; }
__device__ __forceinline__ U128 shl(U128 x, int s)
{
    if (s == 0) return x;
    if (s >= 128) return {0, 0};
    if (s >= 64) return {0, x.lo << (s - 64)};
    return {x.lo << s, (x.hi << s) | (x.lo >> (64 - s))};
}
__device__ __forceinline__ U128 shr(U128 x, int s)
{
    if (s == 0) return x;
    if (s >= 128) return {0, 0};
    if (s >= 64) return {x.hi >> (s - 64), 0};
    return {(x.lo >> s) | (x.hi << (64 - s)), x.hi >> s};
}
__device__ __forceinline__ int popc(u32 x) { return __popc(x); }
__device__ __forceinline__ int popc(u64 x) { return __popcll(x); }
__device__ __forceinline__ int popc(U128 x) { return __popcll(x.lo) + __popcll(x.hi); }
// trailing zeros of a non-zero value
__device__ __forceinline__ int ctz(u32 x) { return __ffs((int)x) - 1; }
__device__ __forceinline__ int ctz(u64 x) { return __ffsll((long long)x) - 1; }
__device__ __forceinline__ int ctz(U128 x) { return x.lo ? ctz(x.lo) : 64 + ctz(x.hi); }
// index of the highest set bit of a non-zero value
__device__ __forceinline__ int msb(u64 x) { return 63 - __clzll((long long)x); }
__device__ __forceinline__ int msb(U128 x) { return x.hi ? 64 + msb(x.hi) : msb(x.lo); }
template <class T> __device__ __forceinline__ T one_at(int p);
template <> __device__ __forceinline__ u32 one_at<u32>(int p) { return 1u << p; }
template <> __device__ __forceinline__ u64 one_at<u64>(int p) { return 1ull << p; }
template <> __device__ __forceinline__ U128 one_at<U128>(int p)
{
    return p >= 64 ? U128{0, 1ull << (p - 64)} : U128{1ull << p, 0};
}
// bits [0, p)
template <class T> __device__ __forceinline__ T mask_below(int p);
template <> __device__ __forceinline__ u32 mask_below<u32>(int p) { return p >= 32 ? ~0u : (1u << p) - 1; }
template <> __device__ __forceinline__ u64 mask_below<u64>(int p) { return p >= 64 ? ~0ull : (1ull << p) - 1; }
template <> __device__ __forceinline__ U128 mask_below<U128>(int p)
{
    if (p >= 128) return {~0ull, ~0ull};
    if (p >= 64) return {~0ull, p == 64 ? 0ull : (1ull << (p - 64)) - 1};
    return {(1ull << p) - 1, 0};
}
__device__ __forceinline__ bool is_zero(u32 x) { return x == 0; }
__device__ __forceinline__ bool is_zero(u64 x) { return x == 0; }
__device__ __forceinline__ bool is_zero(U128 x) { return (x.lo | x.hi) == 0; }

// position of the j-th (0-based) set bit of x (x has more than j set bits)
__device__ __forceinline__ int select64(u64 x, int j)
{
    int s = 0, c;
    c = __popc((u32)x);
    if (j >= c) { j -= c; x >>= 32; s += 32; }
    c = __popc((u32)(x & 0xffffull));
    if (j >= c) { j -= c; x >>= 16; s += 16; }
    c = __popc((u32)(x & 0xffull));
    if (j >= c) { j -= c; x >>= 8; s += 8; }
    c = __popc((u32)(x & 0xfull));
    if (j >= c) { j -= c; x >>= 4; s += 4; }
    c = __popc((u32)(x & 0x3ull));
    if (j >= c) { j -= c; x >>= 2; s += 2; }
    c = (int)(x & 1ull);
    if (j >= c) { s += 1; }
    return s;
}
__device__ __forceinline__ int select(u64 x, int j) { return select64(x, j); }
__device__ __forceinline__ int select(U128 x, int j)
{
    int c = __popcll(x.lo);
    return j < c ? select64(x.lo, j) : 64 + select64(x.hi, j - c);
}

// Select with a byte table: lut[8 v + r] is the position of the r-th set bit
// of the byte v.  Byte-wise popcounts (SWAR) and their prefix sums locate
// the byte that holds the j-th set bit without a search.
__device__ __forceinline__ int select_lut(u32 w, int j, const unsigned char *lut)
{
    u32 c = w - ((w >> 1) & 0x55555555u);
    c = (c & 0x33333333u) + ((c >> 2) & 0x33333333u);
    c = (c + (c >> 4)) & 0x0f0f0f0fu;                       // set bits per byte
    const u32 pre = c * 0x01010101u;                        // byte k: bits in bytes 0..k
    const u32 ge = ((pre | 0x80808080u) - (u32)(j + 1) * 0x01010101u) & 0x80808080u;
    const int b = 4 - __popc(ge);                           // bytes with prefix <= j
    const int before = b == 0 ? 0 : (int)((pre << (32 - 8 * b)) >> 24);
    return 8 * b + lut[((w >> (8 * b)) & 0xffu) * 8 + (u32)(j - before)];
}
__device__ __forceinline__ int select_lut(u64 x, int j, const unsigned char *lut)
{
    const u32 lo = (u32)x;
    const int c = __popc(lo);
    const bool up = j >= c;
    return (up ? 32 : 0) + select_lut(up ? (u32)(x >> 32) : lo, up ? j - c : j, lut);
}
__device__ __forceinline__ int select_lut(U128 x, int j, const unsigned char *lut)
{
    const int c = __popcll(x.lo);
    const bool up = j >= c;
    return (up ? 64 : 0) + select_lut(up ? x.hi : x.lo, up ? j - c : j, lut);
}
// table of select_lut, 2048 bytes
__device__ __forceinline__ unsigned char select_lut_entry(int i)
{
    u32 v = (u32)i >> 3, r = (u32)i & 7;
    for (u32 k = 0; k < r && v; k++) v &= v - 1;  // drop the r lowest set bits
    return v ? (unsigned char)(__ffs((int)v) - 1) : (unsigned char)0;
}

// address word access
__device__ __forceinline__ u64 word0(u64 a) { return a; }
__device__ __forceinline__ u64 word1(u64) { return 0; }
__device__ __forceinline__ u64 word0(U128 a) { return a.lo; }
__device__ __forceinline__ u64 word1(U128 a) { return a.hi; }

template <int W> struct AddrOf;
template <> struct AddrOf<1> {
    typedef u64 T;
    static __device__ __forceinline__ T make(u64 w0, u64) { return w0; }
};
template <> struct AddrOf<2> {
    typedef U128 T;
    static __device__ __forceinline__ T make(u64 w0, u64 w1) { return U128{w0, w1}; }
};

// ---------------------------------------------------------------- hashing

__device__ __forceinline__ u64 mix64(u64 x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}
__device__ __forceinline__ u64 addr_hash(u64 a) { return mix64(a); }
__device__ __forceinline__ u64 addr_hash(U128 a) { return mix64(a.lo ^ mix64(a.hi + 0x9e3779b97f4a7c15ull)); }
// bucket = top log2B bits, LDS slot = low bits
__device__ __forceinline__ u32 bucket_of(u64 h, int log2B) { return log2B == 0 ? 0u : (u32)(h >> (64 - log2B)); }
// 32-bit finalizer (the lowbias32 constants) for addresses of at most 32 bits
__device__ __forceinline__ u32 hash32(u32 x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
// The hash bucket of an address (log2B <= 14): the top log2B bits of a hash
// of the address.  Addresses that fit 32 bits (one word, N + M - 1 <= 32:
// `narrow`, the same for every address of an instance) use the 32-bit
// finalizer, others the 64-bit one.  Any well-mixed function serves: the
// bucket only places an address, and results do not depend on it.
__device__ __forceinline__ u32 bucket_index(u64 a, int log2B, bool narrow)
{
    if (log2B == 0) return 0u;
    return narrow ? hash32((u32)a) >> (32 - log2B) : (u32)(mix64(a) >> (64 - log2B));
}
__device__ __forceinline__ u32 bucket_index(U128 a, int log2B, bool)
{
    return bucket_of(addr_hash(a), log2B);
}

// ---------------------------------------------------------------- Philox

struct R4 {
    u32 x, y, z, w;
};

// a ^ b ^ c in one instruction (gfx950 three-input bit operation, truth
// table 0x96)
__device__ __forceinline__ u32 xor3(u32 a, u32 b, u32 c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }

// Philox4x32-10: ten rounds of the 4x32 S-box with the Weyl key schedule.
__device__ __forceinline__ R4 philox4x32_10(u32 c0, u32 c1, u32 c2, u32 c3, u32 k0, u32 k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        // one 32x32 -> 64 product gives both halves (v_mad_u64_u32)
        const u64 p0 = (u64)0xD2511F53u * c0, p1 = (u64)0xCD9E8D57u * c2;
        const u32 y0 = xor3((u32)(p1 >> 32), c1, k0), y2 = xor3((u32)(p0 >> 32), c3, k1);
        c0 = y0; c1 = (u32)p1; c2 = y2; c3 = (u32)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return R4{c0, c1, c2, c3};
}

// Keying: key = seed ^ address word 1; counter = (address word 0 low/high,
// (tag << 28) | block, step).  tag 0: spawn picks, tag 1: compression.
__device__ __forceinline__ R4 draw(u64 seed, u64 a0, u64 a1, u32 step, u32 tag, u32 block)
{
    u64 k = seed ^ a1;
    return philox4x32_10((u32)a0, (u32)(a0 >> 32), (tag << 28) | block, step, (u32)k, (u32)(k >> 32));
}
__device__ __forceinline__ u32 rword(const R4 &r, int i)
{
    return i == 0 ? r.x : i == 1 ? r.y : i == 2 ? r.z : r.w;
}
// uniform integer in [0, m): floor(r m / 2^32)
__device__ __forceinline__ u32 pick(u32 r, u32 m) { return (u32)(((u64)r * (u64)m) >> 32); }

// ---------------------------------------------------------------- exact sums

constexpr int FIX_FRAC = 80;  // fractional bits of the fixed-point accumulators

// double -> two's complement 128-bit round(v * 2^80) (half-even).  Sets ovf
// when |v| >= 2^46 or v is not finite, and inx when the value is not a
// multiple of 2^-80 (it was rounded; only possible for |v| < 2^-27), so that
// a sum of such values is no longer the exactly rounded sum.
__device__ __forceinline__ void to_fixed(double v, u64 &lo, u64 &hi, int &ovf, int &inx)
{
    u64 b = dbits(v);
    {
        // the common range 2^-27 <= |v| < 2^36 (the mantissa moves up by 1..63
        // bits): exact, a 128-bit shift and a conditional negation.  Taken
        // when every active lane of the wave is in it, so that no lane runs
        // both forms; the general form below gives the same result there.
        const u32 e0 = (u32)(b >> 52) & 0x7ffu;
        if (__all(e0 - 996u < 63u)) {
            const u64 m0 = (b & 0x000FFFFFFFFFFFFFull) | (1ull << 52);
            const int s0 = (int)e0 - 995;
            const u64 L0 = m0 << s0, H0 = m0 >> (64 - s0);
            const u64 neg = b >> 63, sgn = 0ull - neg;
            const u64 lx = L0 ^ sgn;
            lo = lx + neg;
            hi = (H0 ^ sgn) + (lo < lx ? 1ull : 0ull);
            return;
        }
    }
    int e = (int)((b >> 52) & 0x7ff);
    u64 m = b & 0x000FFFFFFFFFFFFFull;
    if (e == 0x7ff) { ovf = 1; lo = hi = 0; return; }
    if (e == 0) { e = 1; } else { m |= 1ull << 52; }
    int sh = e - 1075 + FIX_FRAC;  // value = m 2^(e-1075)
    u64 L, H;
    if (sh >= 0) {
        if (sh > 126 - 53 - 1) { ovf = 1; lo = hi = 0; return; }
        if (sh >= 64) { L = 0; H = m << (sh - 64); }
        else if (sh == 0) { L = m; H = 0; }
        else { L = m << sh; H = m >> (64 - sh); }
    } else {
        int s = -sh;
        if (s > 53) {
            L = 0;
            inx |= m != 0 ? 1 : 0;
        } else {
            u64 q = m >> s, rem = m & ((1ull << s) - 1), half = 1ull << (s - 1);
            inx |= rem != 0 ? 1 : 0;
            if (rem > half || (rem == half && (q & 1ull))) q++;
            L = q;
        }
        H = 0;
    }
    if (b >> 63) { L = ~L + 1; H = ~H + (L == 0 ? 1 : 0); }
    lo = L;
    hi = H;
}
__device__ __forceinline__ void to_fixed(double v, u64 &lo, u64 &hi, int &ovf)
{
    int inx = 0;
    to_fixed(v, lo, hi, ovf, inx);
}

// two's complement 128-bit fixed point -> nearest double (half-even)
__device__ __forceinline__ double from_fixed(u64 lo, u64 hi)
{
    {
        // the common range 2^-16 <= |value| < 2^36 (the high word of the
        // magnitude is nonzero and below 2^52): the 53 leading bits come from
        // the two words with one shift each and the rounding remainder lies in
        // the low word.  Taken when every active lane of the wave is in it;
        // the general form below gives the same result there.
        const u64 sg = (u64)((i64)hi >> 63);  // all ones when negative
        const u64 l = (lo ^ sg) - sg;         // the magnitude's words
        const u64 h = (hi ^ sg) + ((sg != 0 && lo == 0) ? 1ull : 0ull);
        if (__all(h != 0 && h < (1ull << 52))) {
            const int s0 = 12 + msb(h);       // bits dropped: 12 .. 63
            u64 mant = (h << (64 - s0)) | (l >> s0);
            const u64 rem = l & ((1ull << s0) - 1), half = 1ull << (s0 - 1);
            mant += (rem > half || (rem == half && (mant & 1ull))) ? 1ull : 0ull;
            const int s1 = mant == (1ull << 53) ? s0 + 1 : s0;
            mant = mant == (1ull << 53) ? mant >> 1 : mant;
            const double r = bitsd(((u64)(s1 + 995) << 52) | (mant & 0x000FFFFFFFFFFFFFull));
            return sg ? -r : r;
        }
    }
    bool neg = (i64)hi < 0;
    if (neg) { lo = ~lo + 1; hi = ~hi + (lo == 0 ? 1 : 0); }
    if ((lo | hi) == 0) return 0.0;
    int p = hi ? 64 + msb(hi) : msb(lo);
    double r;
    if (p <= 52) {
        r = (double)lo * bitsd((u64)(1023 - FIX_FRAC) << 52);
    } else {
        int s = p - 52;  // drop s low bits
        u64 mant, rem_hi, rem_lo, half_hi, half_lo;
        U128 x{lo, hi};
        U128 q = shr(x, s);
        mant = q.lo;
        U128 rem = x & mask_below<U128>(s);
        U128 half = one_at<U128>(s - 1);
        rem_hi = rem.hi; rem_lo = rem.lo; half_hi = half.hi; half_lo = half.lo;
        bool gt = rem_hi > half_hi || (rem_hi == half_hi && rem_lo > half_lo);
        bool eq = rem_hi == half_hi && rem_lo == half_lo;
        if (gt || (eq && (mant & 1ull))) mant++;
        if (mant == (1ull << 53)) { mant >>= 1; s++; }
        u64 ex = (u64)(s - FIX_FRAC + 52 + 1023);
        r = bitsd((ex << 52) | (mant & 0x000FFFFFFFFFFFFFull));
    }
    return neg ? -r : r;
}

// 128-bit accumulate into LDS words (lo with carry detection, then hi)
__device__ __forceinline__ void lds_acc128(u64 *lo_p, u64 *hi_p, u64 lo, u64 hi)
{
    u64 old = atomicAdd((unsigned long long *)lo_p, (unsigned long long)lo);
    u64 carry = (old + lo) < old ? 1ull : 0ull;
    u64 h = hi + carry;
    if (h) atomicAdd((unsigned long long *)hi_p, (unsigned long long)h);
}
__device__ __forceinline__ void glb_acc128(u64 *p2, u64 lo, u64 hi)
{
    u64 old = atomicAdd((unsigned long long *)&p2[0], (unsigned long long)lo);
    u64 carry = (old + lo) < old ? 1ull : 0ull;
    u64 h = hi + carry;
    if (h) atomicAdd((unsigned long long *)&p2[1], (unsigned long long)h);
}
__device__ __forceinline__ void add128(u64 &alo, u64 &ahi, u64 lo, u64 hi)
{
    u64 n = alo + lo;
    ahi += hi + (n < alo ? 1ull : 0ull);
    alo = n;
}

// ---------------------------------------------------------------- det. log

// ln x with the same operation sequence as the CPU oracle:
// x = (1+f) 2^e, 1+f in [sqrt(1/2), sqrt(2)), s = f/(2+f),
// ln(1+f) = f - (f^2/2 - s (f^2/2 + R)), R = sum_{k>=1} 2 s^(2k)/(2k+1).
__device__ __forceinline__ double det_log(double x)
{
    u64 b = dbits(x);
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    double m = bitsd((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > bitsd(0x3FF6A09E667F3BCDull)) { m = m * 0.5; e += 1; }
    double f = m - 1.0;
    double hfsq = (0.5 * f) * f;
    double s = f / (2.0 + f);
    double z = s * s;
    double R = 2.0 / 27.0;
    for (int k = 12; k >= 1; k--) R = R * z + 2.0 / (double)(2 * k + 1);
    R = R * z;
    double lm = f - (hfsq - s * (hfsq + R));
    double de = (double)e;
    return de * bitsd(0x3FE62E42FEE00000ull) + (de * bitsd(0x3DEA39EF35793C76ull) + lm);
}

}  // namespace fq
