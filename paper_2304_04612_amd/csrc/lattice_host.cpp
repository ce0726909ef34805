// Host construction of the FP16 inverse-CDF table used by the Omega generator.
//
// Sec. 3.1 (eq:g-fp-error, eq:RN-range): a Gaussian value stored in FP16 is
// the round-to-nearest image of the exact draw.  The non-negative finite FP16
// values in increasing order are the bit patterns 0, 1, 2, ...; a magnitude
// |g| rounds to pattern t exactly when it lies below the midpoint mu_t
// between patterns t and t+1 and at or above mu_{t-1}.  With a uniform 63-bit
// integer u, the pattern k = #{ t : T_t <= u } with
//     T_t = floor(2^63 * erf(mu_t / sqrt(2)))
// is therefore distributed as |RN16(g)| to within 2^-63 per cell.  The table
// stops at the first t whose threshold equals 2^63 - 1 (t = 18570).
//
// erf is evaluated in IEEE binary128 (libquadmath), whose 113-bit significand
// leaves the floor of a 63-bit scaled value unaffected.  This file is built
// with the host C++ compiler because binary128 is not available in HIP
// device compilation.
#include <quadmath.h>
#include <stdint.h>
#include <string.h>

namespace {

// Exact value of a non-negative finite FP16 bit pattern.
__float128 f16_value(uint32_t bits) {
    uint32_t e = (bits >> 10) & 0x1F;
    uint32_t m = bits & 0x3FF;
    if (e == 0) return ldexpq((__float128)m, -24);
    return ldexpq((__float128)(1024 + m), (int)e - 25);
}

}  // namespace

extern "C" int rpmi_build_f16_thresholds(uint64_t* table, int capacity) {
    const __float128 two63 = ldexpq(1.0Q, 63);
    const __float128 inv_sqrt2 = 1.0Q / sqrtq(2.0Q);
    const uint64_t top = (uint64_t(1) << 63) - 1;
    for (int t = 0; t < capacity && t < 0x7BFF; ++t) {
        __float128 mu = 0.5Q * (f16_value(t) + f16_value(t + 1));
        __float128 v = floorq(two63 * erfq(mu * inv_sqrt2));
        uint64_t T = v >= (__float128)top ? top : (uint64_t)v;
        table[t] = T;
        if (T == top) return t + 1;
    }
    return -1;  // capacity too small
}

// Guide table over the top L = buckets_log2 bits of the 63-bit u (the
// library uses L = 16): guide[b] = #{ t : T_t < b * 2^(63-L) }, b = 0..2^L,
// so that the pattern for u in bucket b lies in
// [guide[b], guide[b+1]] and only that slice of the table is searched.
extern "C" void rpmi_build_guide(const uint64_t* table, int count, uint32_t* guide, int buckets_log2) {
    const int nb = 1 << buckets_log2;
    const int shift = 63 - buckets_log2;
    int t = 0;
    for (int b = 0; b <= nb; ++b) {
        const unsigned __int128 edge = (unsigned __int128)b << shift;
        while (t < count && (unsigned __int128)table[t] < edge) ++t;
        guide[b] = (uint32_t)t;
    }
}
