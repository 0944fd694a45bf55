/* Host replay of the residue arithmetic the CRT kernels use, step for step
 * in the same precisions, against exact integer residues:
 *  1. every |x| <= 2^26 and every modulus: the quotient from one float FMA
 *     with 1.5 * 2^23 added (its encoding's low 24 bits are 2^22 + q), the
 *     24-bit multiply-add, and the two unsigned 16-bit corrections give the
 *     symmetric residue as an int8;
 *  2. int32 sums above 2^26 (the product epilogue's long contractions):
 *     the fold (x >> 16)(2^16 mod m) + (x & 0xffff) is congruent to x and
 *     within 2^26, so step 1 applies to it;
 *  3. operands: an integer-valued double |z'| < 2^53 is cut into exact
 *     pieces z2 2^36 + z1 2^18 + z0 and x = z2 c36 + z1 c18 + z0 (symmetric
 *     constants) stays within 2^26 and congruent to z'.
 * Exit status 0 when every case matches. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

static const int mods[15] = {256, 255, 253, 251, 247, 241, 239, 233,
                             229, 227, 223, 217, 211, 199, 197};

static inline int i24(int a) { return (int32_t)((uint32_t)a << 8) >> 8; }
static inline int mul24(int a, int b) {
    return (int)(uint32_t)(uint64_t)((int64_t)i24(a) * (int64_t)i24(b));
}
static inline uint16_t min16(uint16_t a, uint16_t b) { return a < b ? a : b; }
static int sym(int64_t z, int m) {
    int64_t t = z % m;
    if (t < 0) t += m;
    if (t > (m - 1) / 2) t -= m;
    return (int)t;
}
static int symc(int64_t c, int m) { return sym(c, m); }

/* the kernel's reduction of one int32 with |x| <= 2^26 */
static int8_t reduce_small(int x, int m, float inv, int *bad_q) {
    const float qf = fmaf((float)x, inv, 0x1.8p23f);
    if (!(qf >= 0x1p23f && qf < 0x1p24f)) ++*bad_q;
    int w;
    memcpy(&w, &qf, 4);
    const int r = mul24(w, -m) + x;
    const int lo = -(m >> 1);
    uint16_t d = (uint16_t)(r - lo);
    d = min16(d, (uint16_t)(d + m));
    d = min16(d, (uint16_t)(d - m));
    return (int8_t)(uint8_t)(uint16_t)(d + lo);
}

static uint64_t s = 88172645463325252ull;
static uint64_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }

int main(void) {
    long bad = 0;
    const int64_t lim = (int64_t)1 << 26;
    for (int i = 0; i < 15; ++i) {
        const int m = mods[i];
        const float inv = (float)(1.0 / m);
        long b = 0;
#pragma omp parallel for reduction(+ : b) schedule(static)
        for (int64_t xx = -lim; xx <= lim; ++xx) {
            int bq = 0;
            if (reduce_small((int)xx, m, inv, &bq) != (int8_t)sym(xx, m) || bq) ++b;
        }
        if (b) printf("step 1: m=%d, %ld mismatches\n", m, b);
        bad += b;
    }
    for (int i = 0; i < 15; ++i) {
        const int m = mods[i], c16 = (int)((1 << 16) % m);
        for (long k = 0; k < 2000000; ++k) {
            int x;
            if (k < 64) x = (k & 1 ? INT32_MIN : INT32_MAX) + (int)(k >> 1) * (k & 1 ? 1 : -1);
            else x = (int)(uint32_t)rnd();
            const int v = mul24(x >> 16, c16) + (x & 0xffff);
            if (v > lim || v < -lim || sym(v, m) != sym(x, m)) {
                if (bad < 5) printf("step 2: m=%d x=%d v=%d\n", m, x, v);
                ++bad;
            }
        }
    }
    for (int i = 0; i < 15; ++i) {
        const int m = mods[i];
        const int c18 = symc(((int64_t)1 << 18) % m, m), c36 = symc(((int64_t)1 << 36) % m, m);
        for (long k = 0; k < 1000000; ++k) {
            int64_t z;
            switch (k % 4) {
            case 0: z = (int64_t)(rnd() >> 11); break;
            case 1: z = (int64_t)(rnd() >> (11 + rnd() % 50)); break;
            case 2: z = ((int64_t)1 << (rnd() % 53)) + (int64_t)(rnd() % 5) - 2; break;
            default: z = (((int64_t)1 << 53) - 1) - (int64_t)(rnd() % 1000); break;
            }
            if (rnd() & 1) z = -z;
            if (z >= ((int64_t)1 << 53) || z <= -((int64_t)1 << 53)) continue;
            const double zt = (double)z;
            const double h = floor(zt * 0x1p-36), t = fma(-h, 0x1p36, zt);
            const double mid = floor(t * 0x1p-18);
            const int z2 = (int)h, z1 = (int)mid, z0 = (int)fma(-mid, 0x1p18, t);
            const int x = mul24(z1, c18) + (mul24(z2, c36) + z0);
            if (x > lim || x < -lim || sym(x, m) != sym(z, m) || z0 < 0 || z0 >= (1 << 18) ||
                z1 < 0 || z1 >= (1 << 18)) {
                if (bad < 5) printf("step 3: m=%d z=%lld\n", m, (long long)z);
                ++bad;
            }
        }
    }
    printf("%ld mismatches\n", bad);
    return bad != 0;
}
