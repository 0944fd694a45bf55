// crt.hip -- step a2 in a second mixed-precision form: the product from
// residues modulo small pairwise-coprime moduli on the int8 matrix cores,
// combined by the Chinese remainder theorem (the construction of Ozaki,
// Uchino and Imamura's "Ozaki scheme II", written here from its idea).
//
// Every line (row of X, column of Y) is scaled by a power of two from its
// largest magnitude and truncated to an integer of `bits` bits:
//   e    = exponent with 2^(e-1) <= max |z| < 2^e  (0 for a zero line),
//   z'   = trunc(z * 2^(bits - e)),   |z'| < 2^bits,
// so the exact integer product P = X' Y' satisfies |P| < K 2^(2 bits).  With
// moduli m_1..m_L (m_i <= 256, product M > 4 K 2^(2 bits)) the residues
// X'_i = X' mod m_i and Y'_i = Y' mod m_i, taken in the symmetric range
// [-floor(m/2), floor((m-1)/2)], fit int8; each T_i = X'_i Y'_i is one int8
// GEMM with exact int32 accumulation (|T_i| <= K 2^14 < 2^31 for K < 2^17),
// and P mod m_i = T_i mod m_i.  P itself is recovered from its L residues:
//   S = sum_i r_i w_i,  w_i = (M / m_i) * ((M / m_i)^(-1) mod m_i),
//   P = S - M * round(S / M),
// with S and M held exactly as three limbs of 40 bits in FP64 (every limb
// product and sum below 2^53), normalised, and summed into one double.
// Then C = P * 2^(e_g + f_h - 2 bits).
//
// Work: L int8 GEMMs instead of the S (S+1) / 2 digit products of the slice
// form, and one accumulator per output instead of one per diagonal, so the
// workgroup tile is 256 x 256.  For tol = 1e-12 at K = 4096: bits = 42,
// L = 13.
//
// The GEMM: 8 waves of 128 x 64 (4 x 2 blocks of v_mfma_i32_32x32x32_i8,
// 128 accumulator registers), one stage = two k-steps of both operands (32
// KB), four stages in LDS filled by direct-to-LDS loads issued three stages
// ahead; the fragments of the next k-step are read while the current one
// multiplies, and the barrier sits between the two k-steps of a stage.
#include <algorithm>

#include "internal.h"

namespace tcu {
namespace {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kMaxMod = 15;
constexpr int kModuli[kMaxMod] = {256, 255, 253, 251, 247, 241, 239, 233,
                                  229, 227, 223, 217, 211, 199, 197};

struct CrtConsts {
    int L, bits;
    int mi[kMaxMod], c16[kMaxMod];  // m_i and 2^16 mod m_i
    int c18[kMaxMod], c36[kMaxMod]; // 2^18 and 2^36 mod m_i, symmetric (|c| <= 128)
    float inv_f[kMaxMod];           // 1 / m_i rounded to float
    double w[kMaxMod][3];  // w_i = w2 2^80 + w1 2^40 + w0
    double Mp[3];          // M in the same limbs
    double inv_M;          // 1 / M rounded to double
};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// The symmetric residues of four int32 sums as four int8 bytes of one word.
// SMALL: every |x| <= 2^26; otherwise x is first replaced by the congruent
// r1 = (x >> 16)(2^16 mod m) + (x & 0xffff), |r1| < 2^24 (c16 = 2^16 mod m;
// checked exhaustively over all int32 x for each modulus).  Then the
// quotient q, x * (1/m) rounded to an integer in float, is within 0.57 of
// x / m.  It comes from one FMA: adding 1.5 * 2^23 to the product makes
// the rounding land on integers, so the low 24 bits of the sum's encoding
// are 2^22 + q.  The 24-bit multiply-add x - (2^22 + q) m then equals
// r - 2^22 m with r = x - q m within 0.57 m of 0, and 2^22 m vanishes
// modulo 2^16.  The symmetric range follows from d = r - lo (mod 2^16) with
// two unsigned 16-bit minimums, min(d, d + m) then min(d, d - m), on two
// residues per instruction.  (Checked exhaustively for |x| <= 2^26 and
// every modulus.)
template <bool SMALL>
__device__ inline uint32_t sym_mod32x4(const int (&x)[4], int m, int c16, float inv) {
    int r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = SMALL ? x[j] : __mul24(x[j] >> 16, c16) + (x[j] & 0xffff);
        const int q22 = __float_as_int(fmaf((float)v, inv, 0x1.8p23f));  // low 24 bits: 2^22 + q
        r[j] = __mul24(q22, -m) + v;
    }
    const unsigned short lo = (unsigned short)(-(m >> 1)), mm = (unsigned short)m;
    const u16x2 lo2 = {lo, lo}, m2 = {mm, mm};
    u16x2 d01 = u16x2{(unsigned short)r[0], (unsigned short)r[1]} - lo2;
    u16x2 d23 = u16x2{(unsigned short)r[2], (unsigned short)r[3]} - lo2;
    d01 = __builtin_elementwise_min(d01, d01 + m2);
    d23 = __builtin_elementwise_min(d23, d23 + m2);
    d01 = __builtin_elementwise_min(d01, d01 - m2) + lo2;
    d23 = __builtin_elementwise_min(d23, d23 - m2) + lo2;
    // bytes 0 and 2 of each pair: residues 0, 1, 2, 3
    return __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, d23),
                                 __builtin_bit_cast(uint32_t, d01), 0x06040200u);
}

__device__ inline int line_exp(unsigned long long bits) {
    const double mx = __longlong_as_double((long long)bits);
    int e = 0;
    if (mx > 0.0) frexp(mx, &e);
    return e;
}

// residue plane layout (as the slice form): res[i][t / 32][(t % 32) / 16][line][t % 16]
__device__ inline int64_t res_offset(int line, int t, int lines_pad) {
    return (((int64_t)(t >> 5) * 2 + ((t >> 4) & 1)) * lines_pad + line) * 16 + (t & 15);
}

// The truncated integer z' = trunc(z 2^(bits - e)) (|z'| < 2^53) as exact
// FP64 pieces z' = z2 2^36 + z1 2^18 + z0, 0 <= z0, z1 < 2^18, |z2| <= 2^17;
// then x = z2 c36 + z1 c18 + z0 is congruent to z' modulo m with |x| < 2^26
// (|c| <= 128), two 24-bit multiply-adds per modulus, and sym_mod32x4<true>
// gives the residues.
struct Pieces {
    int z2, z1, z0;
};

__device__ inline Pieces pieces(double z, int shift) {
    if (!isfinite(z)) z = 0.0;  // non-finite inputs are flagged by the line maxima
    const double zt = trunc(ldexp(z, shift));
    const double h = floor(zt * 0x1p-36);
    const double t = fma(-h, 0x1p36, zt);  // exact, in [0, 2^36)
    const double mid = floor(t * 0x1p-18);
    return Pieces{(int)h, (int)mid, (int)fma(-mid, 0x1p18, t)};
}

// a * b + c with a and b taken as signed 24-bit integers, one instruction
// (written out because the compiler turns two of them into two multiplies
// and a three-way add); b is wave-uniform
__device__ inline int mad24(int a, int b, int c) {
    int d;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
    return d;
}

// residues modulo m_i of 16 pieces, as one 16-byte vector
__device__ inline uint4 residues16(const Pieces (&p)[16], const CrtConsts &cc, int i) {
    const int m = cc.mi[i], c18 = cc.c18[i], c36 = cc.c36[i];
    const float inv = cc.inv_f[i];
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const Pieces &z = p[4 * q + j];
            x[j] = mad24(z.z1, c18, mad24(z.z2, c36, z.z0));
        }
        w[q] = sym_mod32x4<true>(x, m, 0, inv);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// One workgroup per 64 lines x 64 positions (grid: len_pad / 64, lines_pad /
// 64).  Thread (r, g) = (t % 64, t / 64) owns line l0 + r, positions p0 +
// 16 g .. + 15; a wave's 16-byte residue stores are then one contiguous 1 KB
// run per modulus.

// Lines are rows: the 64 x 64 tile is read row-contiguously (a wave reads
// 512 B of one row per load) into padded LDS, then each thread takes its 16
// positions of one row from there.
__global__ void __launch_bounds__(kThreads)
crt_rows_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld,
                const unsigned long long *__restrict__ maxbits, CrtConsts cc,
                int8_t *__restrict__ out, int lines_pad, int len_pad, int *__restrict__ exps) {
    __shared__ double tile[64][64 + 2];  // [line][position]; the pad spreads lines over banks
    const int p0 = blockIdx.x * 64, l0 = blockIdx.y * 64;
    const int t = threadIdx.x;
    // element offset of this thread's load j, advanced by 4 rows per load
    // (a running 64-bit sum instead of a 64-bit product per load)
    int64_t off = (int64_t)(l0 + (t >> 6)) * ld + p0 + (t & 63);
    const int64_t step = 4 * ld;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int lr = (t >> 6) + 4 * j, pc = t & 63;
        const int row = l0 + lr, c = p0 + pc;
        // every lane loads (element 0 stands in outside the matrix), so the
        // sixteen loads are in flight together instead of one branch each
        const bool in = row < rows && c < cols;
        const double v = Z[in ? off : 0];
        tile[lr][pc] = in ? v : 0.0;
        off += step;
    }
    __syncthreads();
    const int r = t & 63, g = t >> 6;
    const int line = l0 + r;
    const int e = line < rows ? line_exp(maxbits[line]) : 0;
    if (line < rows && blockIdx.x == 0 && g == 0) exps[line] = e;
    Pieces pc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) pc[k] = pieces(tile[r][16 * g + k], cc.bits - e);
    const int64_t plane = (int64_t)lines_pad * len_pad;
    int8_t *o = out + res_offset(line, p0 + 16 * g, lines_pad);
    for (int i = 0; i < cc.L; ++i)
        *reinterpret_cast<uint4 *>(o + (int64_t)i * plane) = residues16(pc, cc, i);
}

// Lines are columns: thread (r, g) reads its column's 16 positions directly
// (for each position the wave reads 512 contiguous bytes of one row).
__global__ void __launch_bounds__(kThreads)
crt_cols_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld,
                const unsigned long long *__restrict__ maxbits, CrtConsts cc,
                int8_t *__restrict__ out, int lines_pad, int len_pad, int *__restrict__ exps) {
    const int p0 = blockIdx.x * 64, l0 = blockIdx.y * 64;
    const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int col = l0 + r;
    const int e = col < cols ? line_exp(maxbits[col]) : 0;
    if (col < cols && blockIdx.x == 0 && g == 0) exps[col] = e;
    Pieces pc[16];
    int64_t off = (int64_t)(p0 + 16 * g) * ld + col;  // advanced by one row per load
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int row = p0 + 16 * g + k;
        pc[k] = pieces((row < rows && col < cols) ? Z[off] : 0.0, cc.bits - e);
        off += ld;
    }
    const int64_t plane = (int64_t)lines_pad * len_pad;
    int8_t *o = out + res_offset(col, p0 + 16 * g, lines_pad);
    for (int i = 0; i < cc.L; ++i)
        *reinterpret_cast<uint4 *>(o + (int64_t)i * plane) = residues16(pc, cc, i);
}

// ------------------------------------------------------- the certificate
// The plan of a mixed-form product is certified cell by cell from a lower
// bound of (|X||Y|)[g,h] computed by one int8 GEMM of "magnitude planes":
//   q = floor(|z| 2^(7 - e)) in [0, 127],  e the line's exponent as above,
// so q 2^(e - 7) <= |z| and D_lo = 2^(e_g + f_h - 14) (Q_X Q_Y)[g,h] <=
// (|X||Y|)[g,h], exactly (power-of-two scalings, exact integer sums).  The
// lines also carry their sums of |z| relative to 2^e, s = sum |z| 2^-e
// (rounded up), which bound the truncation errors (see CertArgs).

// The normalised sum of a line, rounded up: the FP64 sum of at most 2^31
// non-negative terms is within a relative 2^-22 of the exact one, and the
// power-of-two scaling is exact (for sums above the subnormal range).
__device__ inline double shat_of(double sum, int e) { return ldexp(sum, -e) * (1.0 + 0x1p-20); }

// wave-wide maximum of non-negative doubles, then one atomic max per wave
__device__ inline void wave_max_to(double v, unsigned long long *dst) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

__device__ inline int8_t mag_q(double z, int e) {
    if (!isfinite(z)) z = 0.0;  // non-finite inputs are flagged by the line maxima
    return (int8_t)(int)floor(ldexp(fabs(z), 7 - e));
}

__device__ inline uint4 pack16(const int8_t (&q)[16]) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        w[j] = (uint32_t)(uint8_t)q[4 * j] | ((uint32_t)(uint8_t)q[4 * j + 1] << 8) |
               ((uint32_t)(uint8_t)q[4 * j + 2] << 16) | ((uint32_t)(uint8_t)q[4 * j + 3] << 24);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Lines are rows (the tile walk of crt_rows_kernel).  sums[line] is the
// line's sum of |z|; the blocks of the first position tile write shat and
// fold its maximum into *umax.
__global__ void __launch_bounds__(kThreads)
mag_rows_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld,
                const unsigned long long *__restrict__ maxbits, const double *__restrict__ sums,
                double *__restrict__ shat, unsigned long long *umax, int8_t *__restrict__ out,
                int lines_pad) {
    __shared__ double tile[64][64 + 2];
    const int p0 = blockIdx.x * 64, l0 = blockIdx.y * 64;
    const int t = threadIdx.x;
    int64_t off = (int64_t)(l0 + (t >> 6)) * ld + p0 + (t & 63);
    const int64_t step = 4 * ld;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int lr = (t >> 6) + 4 * j, pc = t & 63;
        const bool in = l0 + lr < rows && p0 + pc < cols;
        const double v = Z[in ? off : 0];
        tile[lr][pc] = in ? v : 0.0;
        off += step;
    }
    __syncthreads();
    const int r = t & 63, g = t >> 6;
    const int line = l0 + r;
    const int e = line < rows ? line_exp(maxbits[line]) : 0;
    int8_t q[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) q[k] = mag_q(tile[r][16 * g + k], e);
    *reinterpret_cast<uint4 *>(out + res_offset(line, p0 + 16 * g, lines_pad)) = pack16(q);
    if (blockIdx.x == 0 && g == 0) {
        double sh = 0.0;
        if (line < rows) {
            sh = shat_of(sums[line], e);
            shat[line] = sh;
        }
        wave_max_to(sh, umax);
    }
}

// Lines are columns (the walk of crt_cols_kernel); a column's sum is the sum
// of its `parts` partial sums sums[part * cols + col], added in order.
__global__ void __launch_bounds__(kThreads)
mag_cols_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld,
                const unsigned long long *__restrict__ maxbits, const double *__restrict__ sums,
                int parts, double *__restrict__ shat, unsigned long long *umax,
                int8_t *__restrict__ out, int lines_pad) {
    // consecutive workgroups take consecutive column tiles of the same rows,
    // so the workgroups in flight read long runs of each row
    const int l0 = blockIdx.x * 64, p0 = blockIdx.y * 64;
    const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int col = l0 + r;
    const int e = col < cols ? line_exp(maxbits[col]) : 0;
    int8_t q[16];
    int64_t off = (int64_t)(p0 + 16 * g) * ld + col;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int row = p0 + 16 * g + k;
        q[k] = mag_q((row < rows && col < cols) ? Z[off] : 0.0, e);
        off += ld;
    }
    *reinterpret_cast<uint4 *>(out + res_offset(col, p0 + 16 * g, lines_pad)) = pack16(q);
    if (blockIdx.y == 0 && g == 0) {
        double sh = 0.0;
        if (col < cols) {
            double sm = 0.0;
            for (int p = 0; p < parts; ++p) sm += sums[(int64_t)p * cols + col];
            sh = shat_of(sm, e);
            shat[col] = sh;
        }
        wave_max_to(sh, umax);
    }
}

// Per cell (g, h), with T = (Q_X Q_Y)[g,h] and r = 2^14 (s_g + s_h) (r = 0
// when s_g or s_h is 0: an all-zero line leaves nothing to truncate): the
// truncation of both operands to `b`-bit integers per line (the residue
// form) changes the product by at most 2^(e_g + f_h) 2^-b (s_g + s_h), and
// S digits per line with the digit pairs past the first S anti-diagonals
// dropped (the slice forms) by at most 2^(e_g + f_h) 2^-7S (s_g + s_h +
// (S - 1) K).  Against D_lo = 2^(e_g + f_h - 14) T the cell meets the
// tolerance with
//   residue form:  2^-b r <= tcrt T,
//   digit forms:   2^-7S (r + (S - 1) kterm) <= tdig[S] T,  kterm = 2^14 K,
// where tcrt and tdig[S] are the tolerance less the rounding of the FP64
// combination.  The cell's need is the smallest such b and S; a cell with T
// = 0 but r > 0 cannot be bounded (kNeedUncertified).
// The residue form's need of one cell: the smallest b >= 1 with r <= 2^b u,
// u = tcrt T, read off the exponents and mantissas of r (enlarged past the
// rounding of u) and u: with r = mr 2^er and u = mu 2^eu (mantissas in
// [0.5, 1)), b = er - eu, plus 1 when mr > mu.
__device__ inline uint32_t cert_bits(double r, int T, const CertArgs &ca) {
    if (T <= 0) return r > 0.0 ? kNeedUncertified : 0u;
    if (r <= 0.0) return 0u;
    int er, eu;
    const double mr = frexp(r * (1.0 + 0x1p-40), &er);
    const double mu = frexp(ca.tcrt * (double)T, &eu);
    const int b = er - eu + (mr > mu ? 1 : 0);
    return (uint32_t)min(max(b, 1), (int)kNeedUncertified - 1);
}

// The digit forms' need of one cell: the smallest S in 1..8 with
// 2^-7S (r + (S - 1) kterm) <= tdig[S] T (kNeedUncertified when none).
__device__ inline uint32_t cert_slices(double r, int T, const CertArgs &ca) {
    if (T <= 0) return r > 0.0 ? kNeedUncertified : 0u;
    if (r <= 0.0) return 0u;
    const double dT = (double)T;
    uint32_t ns = kNeedUncertified;
#pragma unroll
    for (int S = TCU_MAX_SLICES; S >= 1; --S)
        if (ldexp(r + (S - 1) * ca.kterm, -7 * S) <= ca.tdig[S] * dT) ns = (uint32_t)S;
    return ns;
}

// ---------------------------------------------------------------- the GEMM
// Tile configuration: a workgroup computes BM x BN outputs with NW waves in a
// 2 x (NW / 2) grid (each wave 128 rows by BN / (NW / 2) columns, i.e. WA = 4
// by WB blocks of 32 x 32) and keeps NS stages of two k-steps in LDS.
template <int BN_, int NW_, int NS_, int WPE_>
struct Cfg {
    static constexpr int BM = 256, BN = BN_, NW = NW_, NS = NS_, WPE = WPE_;
    static constexpr int threads = 64 * NW;
    static constexpr int WA = BM / 2 / 32, WB = BN / (NW / 2) / 32;
    static constexpr int KS = 2 * BM + 2 * BN;      // 16-byte chunks per k-step
    static constexpr int STAGE = 2 * KS;            // chunks per stage
    static constexpr int PX = 2 * BM / 64, PY = 2 * BN / 64;  // 1 KB planes per k-step
    static constexpr int PER_WAVE = 2 * (PX + PY) / NW;
    static_assert(2 * (PX + PY) % NW == 0, "planes must split evenly over the waves");
};
// 256 x 256 tiles, 8 waves, 4 stages of 32 KB (128 KB of LDS, one workgroup
// per CU); for wide outputs 256 x 384 tiles, 8 waves of 128 x 96, 4 stages of
// 40 KB (all 160 KB of the CU's LDS, 256 VGPRs): a third fewer LDS fragment
// reads and operand-panel bytes per MFMA.  Measured: the 2^30-record step
// 1535 against 1586 ms; the narrow tile is faster at 8192^3 (6.72 against
// 7.23 ms for 14 moduli) and 4096^3 (0.82-0.83 against 0.83-0.85 ms,
// certificate 0.10 against 0.12 ms).
using CrtCfg = Cfg<256, 8, 4, 2>;
using CrtCfgWide = Cfg<384, 8, 4, 2>;
static_assert(CrtCfg::NS == CrtCfgWide::NS && CrtCfg::BM == CrtCfgWide::BM,
              "both tile shapes share the plane layout's length padding and row tiles");
// output width from which products use the wide tile
constexpr int kWideTileN = 16384;
// Tiles are numbered in groups GROUP_M tile rows deep, so a run of 32 tiles
// (one per CU of an XCD) spans 8 tile rows and 4 columns: fewer of the wide
// tile's 384-line column panels (measured at the 2^30 step: 1513 ms against
// 1543-1557 ms for runs 4 rows deep; 16 rows deep 1508-1513 ms).
constexpr int NUM_XCD = 8, GROUP_M = 8, RUN = 32;
// k-steps of 32 per unrolled round of the main loop: the contraction length
// of the residue planes is padded to a multiple of this
constexpr int kCrtLenAlign = 64 * CrtCfg::NS;
// k per launch of the residue products (a multiple of kCrtLenAlign): every
// int32 sum of a chunk stays below 32768 * 2^14 = 2^29 in magnitude, and a
// contraction up to 131071 runs in at most four chunks
constexpr int kCrtChunk = 32768;
// workgroups per launch of the residue products, at most (and at least the
// workgroups of one modulus): the moduli of a product are grouped into
// launches of about 64 rounds of workgroups.  Measured at 32768^3, 15 moduli:
// all moduli in one launch per 8192-long chunk of k 462 ms, one modulus per
// launch 442 ms, and with one launch over all of k 428 ms (bands of tile rows
// within a modulus gained nothing more); at 4096^3 one launch of all 14
// moduli 0.81 ms against 0.86 ms one per launch.
constexpr int64_t kCrtLaunchWgs = 16384;
static_assert(kCrtChunk % kCrtLenAlign == 0, "chunks hold whole unrolled rounds");

template <int V>
__device__ inline void wait_vm() {
    static_assert(V >= 0 && V < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((V & 15) | ((V >> 4) << 14) | (7 << 4) | (15 << 8));
}
__device__ inline void barrier_nf() { asm volatile("s_barrier" ::: "memory"); }

// While the matrix cores are kept busy, vector-ALU instructions of every wave
// on the SIMD get few issue slots (measured on gfx950: a load whose address
// takes one VALU instruction issued at about a third of its rate beside a
// stream of int8 MFMAs).  The main loop therefore holds no VALU work: each
// load is a direct-to-LDS load whose address is a uniform SGPR base plus the
// lane's fixed byte offset (the SADDR form), with its LDS address in M0,
// both from scalar arithmetic.
__device__ inline void load_lds16(const int8_t *sbase, unsigned voff, unsigned lds_addr) {
    asm volatile("global_load_lds_dwordx4 %0, %1" : : "v"(voff), "s"(sbase), "{m0}"(lds_addr)
                 : "memory");
}

// A uniform value computed on the vector ALU (64-bit products are) moved to
// scalar registers, so that arithmetic on it stays scalar.
__device__ inline const int8_t *to_sgpr(const int8_t *p) {
    const uint64_t u = (uint64_t)(uintptr_t)p;
    // the builtin returns int: widen through uint32_t (zero-extend), or the
    // low word's bit 31 would spill into the high word
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((unsigned)u);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    const uint64_t s = lo | (hi << 32);
    return (const int8_t *)(uintptr_t)s;
}

// The wave's share of one stage's loads: chunk j of the stage is 1 KB (64
// lines x 16 bytes) of operand plane (k-step s, half h) at line block lb.
// Everything here is uniform.
template <typename G>
struct StageLoads {
    const int8_t *src[G::PER_WAVE];  // address of the chunk in stage 0
    int64_t step[G::PER_WAVE];       // bytes from one stage to the next
    unsigned dst[G::PER_WAVE];       // byte offset inside a stage buffer
};

template <typename G>
__device__ inline StageLoads<G> stage_loads(int wave, const int8_t *xi, int xlp, int m0,
                                            const int8_t *yi, int ylp, int n0) {
    StageLoads<G> L;
#pragma unroll
    for (int j = 0; j < G::PER_WAVE; ++j) {
        const int q = wave + G::NW * j;
        const int s = q / (G::PX + G::PY), r = q % (G::PX + G::PY);
        if (r < G::PX) {
            const int h = r / (G::BM / 64), lb = r % (G::BM / 64);
            L.src[j] = xi + (((int64_t)s * 2 + h) * xlp + m0 + lb * 64) * 16;
            L.step[j] = (int64_t)4 * xlp * 16;
            L.dst[j] = (unsigned)(s * G::KS + h * G::BM + lb * 64) * 16u;
        } else {
            const int r2 = r - G::PX;
            const int h = r2 / (G::BN / 64), lb = r2 % (G::BN / 64);
            L.src[j] = yi + (((int64_t)s * 2 + h) * ylp + n0 + lb * 64) * 16;
            L.step[j] = (int64_t)4 * ylp * 16;
            L.dst[j] = (unsigned)(s * G::KS + 2 * G::BM + h * G::BN + lb * 64) * 16u;
        }
        L.src[j] = to_sgpr(L.src[j]);
    }
    return L;
}

template <typename G>
__device__ inline void issue(const StageLoads<G> &L, int st, unsigned buf_addr, unsigned voff) {
#pragma unroll
    for (int j = 0; j < G::PER_WAVE; ++j)
        load_lds16(L.src[j] + (int64_t)st * L.step[j], voff, buf_addr + L.dst[j]);
}

template <int WA, int WB>
struct Frag {
    i4 a[WA], b[WB];
};

// Fragments of k-step S of stage buffer B: fixed per-lane bases plus
// compile-time offsets (the reads need no address arithmetic in the loop).
template <typename G, int B, int S>
__device__ inline void read_frag(const i4 *lds_a, const i4 *lds_b, Frag<G::WA, G::WB> &f) {
#pragma unroll
    for (int a = 0; a < G::WA; ++a) f.a[a] = lds_a[B * G::STAGE + S * G::KS + a * 32];
#pragma unroll
    for (int b = 0; b < G::WB; ++b) f.b[b] = lds_b[B * G::STAGE + S * G::KS + b * 32];
}

// Half H of one k-step's products: row blocks [H WA / 2, (H + 1) WA / 2).
template <int H, int WA, int WB>
__device__ inline void mma_half(const Frag<WA, WB> &f, i16v (&acc)[WA][WB]) {
#pragma unroll
    for (int a = H * WA / 2; a < (H + 1) * WA / 2; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(f.a[a], f.b[b], acc[a][b], 0, 0, 0);
}

// The products of one k-step (fragments f) and the LDS reads of the next
// k-step's fragments (into nf, from k-step S of stage buffer RB); with
// LOADS, also the global-to-LDS loads of stage `ist` into buffer `buf`.
// IL: MFMA i, then load i and read i (while there are any), MFMA by MFMA,
// so every read and load is issued while the matrix pipe has work queued
// (measured on the residue products at 32768^3, 14 moduli: 364-367 against
// 376-379 ms with the reads alone interleaved, MFMA first; 0.7% less again
// with the loads interleaved too; 0.796-0.802 against 0.807-0.828 ms at
// 4096^3).  Otherwise the reads go between the two halves of the MFMAs: the
// certificate's epilogue needs the registers that the interleaved order
// keeps live (with it, it spilled).
template <typename G, int RB, int S, bool IL, bool LOADS>
__device__ inline void kstep(const Frag<G::WA, G::WB> &f, Frag<G::WA, G::WB> &nf,
                             const i4 *lds_a, const i4 *lds_b, i16v (&acc)[G::WA][G::WB],
                             const StageLoads<G> &L, int ist, unsigned buf, unsigned voff) {
    constexpr int WA = G::WA, WB = G::WB, PW = G::PER_WAVE;
    if constexpr (IL) {
        static_assert(WA * WB >= WA + WB && WA * WB >= PW, "too few MFMAs to interleave");
#pragma unroll
        for (int i = 0; i < WA * WB; ++i) {
            acc[i / WB][i % WB] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                f.a[i / WB], f.b[i % WB], acc[i / WB][i % WB], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (LOADS) {
                if (i < PW) load_lds16(L.src[i] + (int64_t)ist * L.step[i], voff, buf + L.dst[i]);
            }
            if (i < WA)
                nf.a[i] = lds_a[RB * G::STAGE + S * G::KS + i * 32];
            else if (i < WA + WB)
                nf.b[i - WA] = lds_b[RB * G::STAGE + S * G::KS + (i - WA) * 32];
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        if constexpr (LOADS) {
            issue<G>(L, ist, buf, voff);
            __builtin_amdgcn_sched_barrier(0);
        }
        mma_half<0>(f, acc);
        __builtin_amdgcn_sched_barrier(0);
        read_frag<G, RB, S>(lds_a, lds_b, nf);
        __builtin_amdgcn_sched_barrier(0);
        mma_half<1>(f, acc);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// One stage of the main loop, stage index st held in buffer B.  fc holds
// the fragments of its first k-step.  The second k-step's fragments (fm) are
// read during the first k-step's MFMAs, the next stage's first k-step (into
// fc) during the second's, so every LDS read has matrix work to land behind.
// Every stage issues one stage of loads (the last ones repeat stage nst - 1
// into buffers no wave reads any more), so "stage st + 1 has landed" is
// always "at most NS - 3 later stages in flight".
template <typename G, int B, bool IL>
__device__ inline void crt_stage(int st, int nst, const StageLoads<G> &L, unsigned lds_addr,
                                 unsigned voff, const i4 *lds_a, const i4 *lds_b,
                                 Frag<G::WA, G::WB> &fc, Frag<G::WA, G::WB> &fm,
                                 i16v (&acc)[G::WA][G::WB]) {
    constexpr int NS = G::NS, PW = G::PER_WAVE;
    kstep<G, B, 1, IL, false>(fc, fm, lds_a, lds_b, acc, L, 0, 0u, voff);
    wait_vm<(NS - 3) * PW>();
    barrier_nf();
    const int ist = st + NS - 1 < nst ? st + NS - 1 : nst - 1;
    kstep<G, (B + 1) % NS, 0, IL, true>(fm, fc, lds_a, lds_b, acc, L, ist,
                                        lds_addr + (unsigned)((B + NS - 1) % NS) * G::STAGE * 16u,
                                        voff);
}

template <typename G, int B, bool IL>
__device__ inline void crt_stages(int st, int nst, const StageLoads<G> &L, unsigned lds_addr,
                                  unsigned voff, const i4 *lds_a, const i4 *lds_b,
                                  Frag<G::WA, G::WB> &fc, Frag<G::WA, G::WB> &fm,
                                  i16v (&acc)[G::WA][G::WB]) {
    crt_stage<G, B, IL>(st + B, nst, L, lds_addr, voff, lds_a, lds_b, fc, fm, acc);
    if constexpr (B + 1 < G::NS)
        crt_stages<G, B + 1, IL>(st, nst, L, lds_addr, voff, lds_a, lds_b, fc, fm, acc);
}

// What the int8 GEMM does with its exact int32 sums.
constexpr int kEpiResidue = 0;  // residues modulo the workgroup's modulus, int8 planes
constexpr int kEpiCertify = 1;  // the residue form's per-cell needs (cert_bits), maximum into ca
constexpr int kEpiCertifyDigits = 3;  // the digit forms' (cert_slices)
constexpr int kEpiCount = 2;    // the int32 sums themselves (pair counts), into cnt

// nblk (k-steps) must be a multiple of 2 NS.  SMALL: nblk * 32 <= 4096, so
// every int32 sum is at most 2^26 in magnitude (and no carry).  carry: this
// launch is a later chunk of a longer contraction, whose earlier chunks'
// residues it adds to its own sums before reducing them (only !SMALL).
template <typename G, bool SMALL, int EPI>
__global__ void __launch_bounds__(G::threads) __attribute__((amdgpu_waves_per_eu(G::WPE, G::WPE)))
gemm_crt_kernel(int m, int n, int nblk, int tiles_m, int tiles_n, const int8_t *__restrict__ xs,
                int xlp, const int8_t *__restrict__ ys, int ylp, int64_t plane_x,
                int64_t plane_y, CrtConsts cc, int8_t *__restrict__ res, int64_t plane_res,
                CertArgs ca, int32_t *__restrict__ cnt, int64_t ldcnt, int carry) {
    constexpr int WA = G::WA, WB = G::WB, PW = G::PER_WAVE, NS = G::NS;
    __shared__ __attribute__((aligned(16))) i4 lds[NS * G::STAGE];
    // workgroup -> (modulus, tile).  Tiles of one modulus are numbered in
    // groups GROUP_M tile-rows deep.  Workgroups go to the XCDs round robin;
    // when the count allows, the j-th workgroup of XCD x takes run
    // (j / 32) * NUM_XCD + x of 32 consecutive tiles, so at any time the
    // eight XCDs work on neighbouring runs of one modulus (each XCD's L2
    // reuses its run's panels; their misses meet in the shared last-level
    // cache); otherwise each XCD takes one contiguous share.
    const int tiles = tiles_m * tiles_n;
    const int total = tiles * cc.L;
    const int wg = blockIdx.x;
    const int x = wg % NUM_XCD, j = wg / NUM_XCD;
    int logical = wg;
    if (total % (NUM_XCD * RUN) == 0) {
        logical = ((j / RUN) * NUM_XCD + x) * RUN + j % RUN;
    } else {
        const int per = total / NUM_XCD;
        if (wg < per * NUM_XCD) logical = x * per + j;
    }
    const int mod = logical / tiles;
    const int t = logical % tiles;
    const int group = GROUP_M * tiles_n;
    const int first_m = (t / group) * GROUP_M;
    const int gm = min(tiles_m - first_m, GROUP_M);
    const int tm = first_m + (t % group) % gm, tn = (t % group) / gm;
    const int m0 = tm * G::BM, n0 = tn * G::BN;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int l32 = lane & 31, half = lane >> 5;
    const unsigned voff = (unsigned)lane * 16u;
    const unsigned lds_addr = (unsigned)(uintptr_t)lds;
    const i4 *lds_a = lds + half * G::BM + wm * 32 * WA + l32;
    const i4 *lds_b = lds + 2 * G::BM + half * G::BN + wn * 32 * WB + l32;
    const StageLoads<G> L = stage_loads<G>(wave, xs + (int64_t)mod * plane_x, xlp, m0,
                                           ys + (int64_t)mod * plane_y, ylp, n0);

    i16v acc[WA][WB];
#pragma unroll
    for (int a = 0; a < WA; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) acc[a][b] = i16v{};

    const int nst = nblk / 2;
    // prologue: stages 0 .. NS-2 in flight (repeating the last stage when
    // there are fewer), fragments of k-step 0
#pragma unroll
    for (int st = 0; st < NS - 1; ++st)
        issue<G>(L, st < nst ? st : nst - 1, lds_addr + (unsigned)st * G::STAGE * 16u, voff);
    wait_vm<(NS - 2) * PW>();
    barrier_nf();
    Frag<WA, WB> fc, fm;
    read_frag<G, 0, 0>(lds_a, lds_b, fc);
    for (int st = 0; st < nst; st += NS)
        crt_stages<G, 0, EPI == kEpiResidue>(st, nst, L, lds_addr, voff, lds_a, lds_b, fc, fm,
                                             acc);
    wait_vm<0>();  // no load into LDS outlives the loop

    if constexpr (EPI == kEpiCount) {
#pragma unroll
        for (int a = 0; a < WA; ++a) {
            const int rbase = m0 + wm * 32 * WA + a * 32;
            if (rbase >= m) continue;
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                const int col = n0 + wn * 32 * WB + b * 32 + l32;
                if (col >= n) continue;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int row = rbase + 8 * (i >> 2) + 4 * half + (i & 3);
                    if (row < m) cnt[(int64_t)row * ldcnt + col] = acc[a][b][i];
                }
            }
        }
        return;
    }
    if constexpr (EPI == kEpiCertify || EPI == kEpiCertifyDigits) {
        // each cell's need; the wave's maxima go out in one atomic each.  The
        // residue form also stores every cell's need (one byte, in the
        // residues' order: one 16-byte store per lane and 32 x 32 block), and
        // the largest and the smallest nonzero need among the cells the
        // certificate bounds.
        uint32_t need = 0, cneed = 0, mneed = kNeedUncertified;
#pragma unroll
        for (int a = 0; a < WA; ++a) {
            const int rbase = m0 + wm * 32 * WA + a * 32;
            if (rbase >= m) continue;
#pragma unroll
            for (int b = 0; b < WB; ++b) {
                const int col = n0 + wn * 32 * WB + b * 32 + l32;
                if (col >= n) continue;
                const double sy = ca.sy[col];
                uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int row = rbase + 8 * (i >> 2) + 4 * half + (i & 3);
                    if (row >= m) continue;
                    // an all-zero line makes every term of the cell zero
                    // in the exact and in the truncated product alike
                    const double sx = ca.sx[row];
                    const double r = (sx > 0.0 && sy > 0.0) ? 16384.0 * (sx + sy) : 0.0;
                    const uint32_t c = EPI == kEpiCertify ? cert_bits(r, acc[a][b][i], ca)
                                                          : cert_slices(r, acc[a][b][i], ca);
                    need = max(need, c);
                    if (c < kNeedUncertified) cneed = max(cneed, c);
                    if (c > 0) mneed = min(mneed, c);
                    w[i >> 2] |= c << (8 * (i & 3));
                }
                if (EPI == kEpiCertify && ca.need_plane != nullptr)
                    *reinterpret_cast<uint4 *>(ca.need_plane +
                                               ((int64_t)(rbase >> 5) * n + col) * 32 + 16 * half) =
                        make_uint4(w[0], w[1], w[2], w[3]);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            need = max(need, (uint32_t)__shfl_xor((int)need, off));
            cneed = max(cneed, (uint32_t)__shfl_xor((int)cneed, off));
            mneed = min(mneed, (uint32_t)__shfl_xor((int)mneed, off));
        }
        // Every workgroup of the launch ends here at about the same time, and
        // same-address atomics from all of them serialise.  The waves' values
        // meet in LDS (free once every wave has left the main loop), and the
        // workgroup skips an atomic that would not change the running maximum
        // (or minimum); that value only moves one way, so a stale read can
        // only cause an atomic that was not needed.
        __syncthreads();
        uint32_t *red = reinterpret_cast<uint32_t *>(lds);
        if (lane == 0) {
            red[wave] = need;
            red[G::NW + wave] = cneed;
            red[2 * G::NW + wave] = mneed;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < G::NW; ++w) {
                need = max(need, red[w]);
                cneed = max(cneed, red[G::NW + w]);
                mneed = min(mneed, red[2 * G::NW + w]);
            }
            uint32_t *nb = EPI == kEpiCertify ? ca.need_bits : ca.need_slices;
            if (need > __atomic_load_n(nb, __ATOMIC_RELAXED)) atomicMax(nb, need);
            if (EPI == kEpiCertify && ca.need_cert != nullptr &&
                cneed > __atomic_load_n(ca.need_cert, __ATOMIC_RELAXED))
                atomicMax(ca.need_cert, cneed);
            if (EPI == kEpiCertify && ca.need_min != nullptr && mneed < kNeedUncertified &&
                mneed < __atomic_load_n(ca.need_min, __ATOMIC_RELAXED))
                atomicMin(ca.need_min, mneed);
        }
        return;
    }
    // epilogue: residues of the int32 sums as int8 in the accumulator's own
    // order (see crt_reconstruct_kernel): one 16-byte store per 32 x 32 block
    const int mi = cc.mi[mod], c16 = cc.c16[mod];
    const float inv = cc.inv_f[mod];
    int8_t *r = res + (int64_t)mod * plane_res;
#pragma unroll
    for (int a = 0; a < WA; ++a) {
        const int rb = (m0 + wm * 32 * WA + a * 32) >> 5;
        if (rb * 32 >= m) continue;
#pragma unroll
        for (int b = 0; b < WB; ++b) {
            const int col = n0 + wn * 32 * WB + b * 32 + l32;
            if (col >= n) continue;
            uint4 *dst = reinterpret_cast<uint4 *>(r + ((int64_t)rb * n + col) * 32 + 16 * half);
            // a later chunk of the contraction adds the residues the earlier
            // chunks left (congruent to their sums), byte j of word q for sum 4q + j
            uint32_t prev[4] = {0u, 0u, 0u, 0u};
            if (!SMALL && carry) {
                const uint4 p4 = *dst;
                prev[0] = p4.x; prev[1] = p4.y; prev[2] = p4.z; prev[3] = p4.w;
            }
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int xs4[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    xs4[j] = acc[a][b][4 * q + j] + (int)(int8_t)(prev[q] >> (8 * j));
                w[q] = sym_mod32x4<SMALL>(xs4, mi, c16, inv);
            }
            *dst = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

// --------------------------------------------------------- reconstruction
constexpr double kLimb = 1099511627776.0;  // 2^40

// P from S = s2 2^80 + s1 2^40 + s0 (exact limb sums of r_i w_i):
// q = round(S / M), the limbs of S - q M exactly, balanced carries (|p0|,
// |p1| <= 2^39, so the sum rounds only at the end), one double.  The plan
// keeps |P| < M / (2 (1 + 2^-38)), so S / M lies within 1/2 - 2^-39 of the
// integer q, and |S / M| < 15 * 128 < 2^11.  Each of the two roundings of
// sd is below 2^-42 M (the inner one only matters when M >= 2^80, and then
// |s1| 2^40 < 1920 M), and the rounded reciprocal and the product add at
// most 2 * 2^-53 * 2^11 relative to 1: sd * (1/M) lies within 2^-40 of
// S / M and rounds to the same q.
__device__ inline double crt_finish(double s0, double s1, double s2, const CrtConsts &cc) {
    const double sd = fma(s2, kLimb * kLimb, fma(s1, kLimb, s0));
    const double q = rint(sd * cc.inv_M);
    double p0 = fma(-q, cc.Mp[0], s0), p1 = fma(-q, cc.Mp[1], s1), p2 = fma(-q, cc.Mp[2], s2);
    double c = rint(p0 * (1.0 / kLimb));
    p0 = fma(-c, kLimb, p0);
    p1 += c;
    c = rint(p1 * (1.0 / kLimb));
    p1 = fma(-c, kLimb, p1);
    p2 += c;
    return fma(p2, kLimb * kLimb, fma(p1, kLimb, p0));
}

// Residue layout: res[i][row / 32][col][p], p = 16 ((row % 8) / 4) + 4 ((row %
// 32) / 8) + row % 4 -- the order in which one lane of the int8 MFMA holds a
// column of its 32 x 32 block.  A thread takes 8 bytes (8 rows of one column:
// rows 32 rb + 8 j + 4 h + (0..3) for j = 2 (q % 2) + (0, 1), h = q / 2) from
// each modulus plane; a wave reads 512 contiguous bytes per modulus.  The
// modulus count L is a template argument, so that both loops over the
// planes unroll fully and the residues stay in fixed registers.
template <int L>
__global__ void __launch_bounds__(kThreads)
crt_reconstruct_kernel(int m, int n, const int8_t *__restrict__ res, int64_t plane, CrtConsts cc,
                       const int *__restrict__ ex, const int *__restrict__ ey,
                       double *__restrict__ C, int64_t ldc, int accumulate) {
    const int col = blockIdx.x * (kThreads / 4) + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    const int rb = blockIdx.y;
    if (col >= n) return;
    const int8_t *base = res + ((int64_t)rb * n + col) * 32 + 8 * q;
    double s[8][3];
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j][0] = s[j][1] = s[j][2] = 0.0;
    // all of this thread's residue loads first (independent, in flight
    // together)
    uint2 vr[L];
#pragma unroll
    for (int i = 0; i < L; ++i) vr[i] = *reinterpret_cast<const uint2 *>(base + (int64_t)i * plane);
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint2 v = vr[i];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const double r = (double)(int8_t)((j < 4 ? v.x : v.y) >> (8 * (j & 3)));
            s[j][0] = fma(r, cc.w[i][0], s[j][0]);  // exact: |r w| < 2^47, sums < 2^51
            s[j][1] = fma(r, cc.w[i][1], s[j][1]);
            s[j][2] = fma(r, cc.w[i][2], s[j][2]);
        }
    }
    const int ec = ey[col] - 2 * cc.bits;
    const int row0 = 32 * rb + 16 * (q & 1) + 4 * (q >> 1);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int row = row0 + 8 * (j >> 2) + (j & 3);
        if (row < m) {
            const double v = ldexp(crt_finish(s[j][0], s[j][1], s[j][2], cc), ex[row] + ec);
            double *dst = C + (int64_t)row * ldc + col;
            *dst = accumulate ? *dst + v : v;
        }
    }
}

typedef void (*ReconstructLaunch)(dim3, hipStream_t, int, int, const int8_t *, int64_t,
                                  const CrtConsts &, const int *, const int *, double *, int64_t,
                                  int);

template <int L>
void reconstruct_launch(dim3 grid, hipStream_t s, int m, int n, const int8_t *res, int64_t plane,
                        const CrtConsts &cc, const int *ex, const int *ey, double *C, int64_t ldc,
                        int accumulate) {
    crt_reconstruct_kernel<L><<<grid, kThreads, 0, s>>>(m, n, res, plane, cc, ex, ey, C, ldc,
                                                        accumulate);
}

// indexed by the modulus count, 1 .. kMaxMod
constexpr ReconstructLaunch kReconstruct[kMaxMod + 1] = {
    nullptr,
    reconstruct_launch<1>,  reconstruct_launch<2>,  reconstruct_launch<3>,  reconstruct_launch<4>,
    reconstruct_launch<5>,  reconstruct_launch<6>,  reconstruct_launch<7>,  reconstruct_launch<8>,
    reconstruct_launch<9>,  reconstruct_launch<10>, reconstruct_launch<11>, reconstruct_launch<12>,
    reconstruct_launch<13>, reconstruct_launch<14>, reconstruct_launch<15>};
static_assert(kMaxMod == 15, "one reconstruction instance per modulus count");

// ------------------------------------------------------------- host side
typedef unsigned __int128 u128;

int inv_mod(int a, int m) {  // a^(-1) mod m, gcd(a, m) = 1
    int t = 0, nt = 1, r = m, nr = a % m;
    while (nr != 0) {
        const int q = r / nr;
        int tmp = t - q * nt;
        t = nt;
        nt = tmp;
        tmp = r - q * nr;
        r = nr;
        nr = tmp;
    }
    return t < 0 ? t + m : t;
}

CrtConsts make_consts(int L, int bits) {
    CrtConsts cc{};
    cc.L = L;
    cc.bits = bits;
    u128 M = 1;
    for (int i = 0; i < L; ++i) M *= (u128)kModuli[i];
    const u128 mask = ((u128)1 << 40) - 1;
    for (int i = 0; i < L; ++i) {
        const int mi = kModuli[i];
        cc.mi[i] = mi;
        cc.c16[i] = 65536 % mi;
        const int c18 = (int)((1ull << 18) % (unsigned long long)mi);
        const int c36 = (int)((1ull << 36) % (unsigned long long)mi);
        cc.c18[i] = c18 > mi / 2 ? c18 - mi : c18;
        cc.c36[i] = c36 > mi / 2 ? c36 - mi : c36;
        cc.inv_f[i] = (float)(1.0 / mi);
        const u128 Mi = M / (u128)mi;
        const int yi = inv_mod((int)(Mi % (u128)mi), mi);
        const u128 w = Mi * (u128)yi;  // < M
        cc.w[i][0] = (double)(uint64_t)(w & mask);
        cc.w[i][1] = (double)(uint64_t)((w >> 40) & mask);
        cc.w[i][2] = (double)(uint64_t)(w >> 80);
    }
    cc.Mp[0] = (double)(uint64_t)(M & mask);
    cc.Mp[1] = (double)(uint64_t)((M >> 40) & mask);
    cc.Mp[2] = (double)(uint64_t)(M >> 80);
    cc.inv_M = 1.0 / (double)M;
    return cc;
}

}  // namespace

double crt_modulus_bits(int L) {
    double b = 0.0;
    for (int i = 0; i < L && i < kMaxMod; ++i) b += log2((double)kModuli[i]);
    return b;
}

int crt_max_moduli() { return kMaxMod; }

int64_t crt_residue_plane(int64_t m, int64_t n) { return (m + 31) / 32 * 32 * n; }

int crt_len_align() { return kCrtLenAlign; }
int crt_tile_cols(int64_t n) { return n >= kWideTileN ? CrtCfgWide::BN : CrtCfg::BN; }

hipError_t launch_crt_split(const double *Z, int rows, int cols, int64_t ld, int axis,
                            const unsigned long long *maxbits, int L, int bits, int8_t *out,
                            int lines_pad, int len_pad, int *exps, hipStream_t s) {
    // the row kernel reads element 0 in place of positions outside the matrix
    if (rows < 1 || cols < 1 || lines_pad % 64 || len_pad % 64) return hipErrorInvalidValue;
    const CrtConsts cc = make_consts(L, bits);
    const dim3 grid((unsigned)(len_pad / 64), (unsigned)(lines_pad / 64));
    if (axis == 0)
        crt_rows_kernel<<<grid, kThreads, 0, s>>>(Z, rows, cols, ld, maxbits, cc, out, lines_pad,
                                                  len_pad, exps);
    else
        crt_cols_kernel<<<grid, kThreads, 0, s>>>(Z, rows, cols, ld, maxbits, cc, out, lines_pad,
                                                  len_pad, exps);
    return hipGetLastError();
}

namespace {

// The residue products on tile shape G (see launch_gemm_crt).
template <typename G>
hipError_t gemm_crt_launches(int m, int n, int k, const CrtConsts &cc, const int8_t *xs,
                             int x_lines_pad, const int8_t *ys, int y_lines_pad, int len_pad,
                             int8_t *res, int64_t plane_res, hipStream_t s) {
    const int L = cc.L;
    const int tiles_m = (m + G::BM - 1) / G::BM, tiles_n = (n + G::BN - 1) / G::BN;
    const CertArgs none{};
    const int64_t px = (int64_t)x_lines_pad * len_pad, py = (int64_t)y_lines_pad * len_pad;
    hipError_t e = hipSuccess;
    // The workgroups of one launch start together and stream the same
    // k-slices of shared panels, but drift apart in k over the launch's
    // rounds, and the caches then serve each slice to fewer of them.  So a
    // large product runs as one launch per group of moduli; a contraction
    // longer than kCrtChunk as chunks of k, each later chunk adding the
    // residues the earlier ones left.
    const int per = (int)std::max<int64_t>(
        1, std::min<int64_t>(L, kCrtLaunchWgs / ((int64_t)tiles_m * tiles_n)));
    for (int g0 = 0; g0 < L && e == hipSuccess; g0 += per) {
        // moduli [g0, g0 + gn) in one launch per chunk
        const int gn = std::min(per, L - g0);
        CrtConsts cg = cc;
        cg.L = gn;
        for (int i = 0; i < gn; ++i) {
            cg.mi[i] = cc.mi[g0 + i];
            cg.c16[i] = cc.c16[g0 + i];
            cg.inv_f[i] = cc.inv_f[g0 + i];
        }
        const int64_t gw = (int64_t)tiles_m * tiles_n * gn;
        const int8_t *xg = xs + g0 * px, *yg = ys + g0 * py;
        int8_t *rg = res + g0 * plane_res;
        for (int k0 = 0; k0 < len_pad && e == hipSuccess; k0 += kCrtChunk) {
            const int kn = std::min(kCrtChunk, len_pad - k0);
            // a chunk starts k0 / 32 k-steps into each plane: k0 bytes per line
            const int8_t *xc = xg + (int64_t)k0 * x_lines_pad, *yc = yg + (int64_t)k0 * y_lines_pad;
            // |sum| <= kn 2^14 (residues at most 128 in magnitude)
            if (kn <= 4096 && k0 == 0)
                gemm_crt_kernel<G, true, kEpiResidue><<<(unsigned)gw, G::threads, 0, s>>>(
                    m, n, kn / 32, tiles_m, tiles_n, xc, x_lines_pad, yc, y_lines_pad, px, py,
                    cg, rg, plane_res, none, nullptr, 0, 0);
            else
                gemm_crt_kernel<G, false, kEpiResidue><<<(unsigned)gw, G::threads, 0, s>>>(
                    m, n, kn / 32, tiles_m, tiles_n, xc, x_lines_pad, yc, y_lines_pad, px, py,
                    cg, rg, plane_res, none, nullptr, 0, k0 > 0 ? 1 : 0);
            e = hipGetLastError();
        }
    }
    return e;
}

// The certificate's or the counts' int8 product on tile shape G.
template <typename G, int EPI>
hipError_t gemm_crt_single(int m, int n, int k, const int8_t *qa, int a_lines_pad,
                           const int8_t *qb, int b_lines_pad, int len_pad, const CertArgs &ca,
                           int32_t *count, int64_t ldc, hipStream_t s) {
    const CrtConsts cc = make_consts(1, 0);
    const int tiles_m = (m + G::BM - 1) / G::BM, tiles_n = (n + G::BN - 1) / G::BN;
    const int64_t pa = (int64_t)a_lines_pad * len_pad, pb = (int64_t)b_lines_pad * len_pad;
    gemm_crt_kernel<G, false, EPI><<<(unsigned)(tiles_m * tiles_n), G::threads, 0, s>>>(
        m, n, len_pad / 32, tiles_m, tiles_n, qa, a_lines_pad, qb, b_lines_pad, pa, pb, cc,
        nullptr, 0, ca, count, ldc, 0);
    return hipGetLastError();
}

// Operand planes fit the tile shape the product of width n uses.
bool crt_planes_ok(int m, int n, int k, int a_lines_pad, int b_lines_pad, int len_pad) {
    return a_lines_pad % CrtCfg::BM == 0 && b_lines_pad % crt_tile_cols(n) == 0 &&
           len_pad % kCrtLenAlign == 0 && len_pad >= k && a_lines_pad >= m && b_lines_pad >= n;
}

}  // namespace

hipError_t launch_gemm_crt(int m, int n, int k, int L, int bits, const int8_t *xs, int x_lines_pad,
                           const int8_t *ys, int y_lines_pad, int len_pad, int8_t *res,
                           const int *ex, const int *ey, double *C, int64_t ldc, int accumulate,
                           hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    if (!crt_planes_ok(m, n, k, x_lines_pad, y_lines_pad, len_pad) || L < 1 || L > kMaxMod)
        return hipErrorInvalidValue;
    const CrtConsts cc = make_consts(L, bits);
    const int64_t plane_res = crt_residue_plane(m, n);
    hipError_t e;
    {
        TraceScope ts(TCU_KERNEL_GEMM_CRT, m, n, k, L, L * 2.0 * m * n * (double)k, s);
        e = crt_tile_cols(n) == CrtCfgWide::BN
                ? gemm_crt_launches<CrtCfgWide>(m, n, k, cc, xs, x_lines_pad, ys, y_lines_pad,
                                                len_pad, res, plane_res, s)
                : gemm_crt_launches<CrtCfg>(m, n, k, cc, xs, x_lines_pad, ys, y_lines_pad,
                                            len_pad, res, plane_res, s);
    }
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((n + kThreads / 4 - 1) / (kThreads / 4)), (unsigned)((m + 31) / 32));
    kReconstruct[L](grid, s, m, n, res, plane_res, cc, ex, ey, C, ldc, accumulate);
    return hipGetLastError();
}

namespace {

// The segment of a cell with this need: the first j with need > t[j]
// (kExcThresholds: none).
__device__ inline int exc_segment(uint32_t need, const ExcThresholds &thr) {
    int seg = kExcThresholds;
#pragma unroll
    for (int j = kExcThresholds - 1; j >= 0; --j)
        if (need > thr.t[j]) seg = j;
    return seg;
}

// The exception scan: one 16-byte chunk of the need plane per lane (half a
// column of a 32-row block, the certificate's store), waves walking the
// plane in step so that a segment's list slots are taken with one atomic
// per wave.  A wave that has to drop cells of a full segment raises the
// segment's count above cap once, so the count then says "overflowed".
__global__ void __launch_bounds__(kThreads)
need_scan_kernel(const uint8_t *__restrict__ plane, int m, int n, ExcThresholds thr,
                 int4 *__restrict__ list, uint32_t cap, StatusBlock *st) {
    const int64_t chunks = (int64_t)((m + 31) / 32) * n * 2;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    bool full[kExcThresholds] = {}, marked[kExcThresholds] = {};
    for (int64_t u0 = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); u0 < chunks;
         u0 += stride) {
        const int64_t u = u0 + lane;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        int row0 = 0, col = 0;
        if (u < chunks) {
            const uint4 v = reinterpret_cast<const uint4 *>(plane)[u];
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
            const int64_t rb = u / (2 * (int64_t)n), rem = u % (2 * (int64_t)n);
            col = (int)(rem >> 1);
            row0 = (int)(rb * 32) + 4 * (int)(rem & 1);
        }
        // segment of each of the lane's 16 cells (kExcThresholds: none)
        uint32_t cnt[kExcThresholds] = {};
        uint32_t any = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t need = (w[i >> 2] >> (8 * (i & 3))) & 255u;
            const int row = row0 + 8 * (i >> 2) + (i & 3);
            const int seg = row < m ? exc_segment(need, thr) : kExcThresholds;
#pragma unroll
            for (int j = 0; j < kExcThresholds; ++j) cnt[j] += seg == j ? 1u : 0u;
            any |= seg < kExcThresholds ? 1u : 0u;
        }
        if (__ballot(any) == 0ull) continue;
#pragma unroll
        for (int j = 0; j < kExcThresholds; ++j) {
            // slots for this wave's cells of segment j: an inclusive scan over the lanes
            uint32_t incl = cnt[j];
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
                if (lane >= off) incl += t;
            }
            const uint32_t total = (uint32_t)__shfl((int)incl, 63);
            if (total == 0) continue;
            if (full[j]) {
                if (!marked[j] && lane == 0) atomicMax(&st->exc_seg[j], cap + 1);
                marked[j] = true;
                continue;
            }
            uint32_t base = 0;
            if (lane == 63) base = atomicAdd(&st->exc_seg[j], total);
            base = (uint32_t)__shfl((int)base, 63);
            full[j] = base + total >= cap;
            uint32_t idx = base + incl - cnt[j];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t need = (w[i >> 2] >> (8 * (i & 3))) & 255u;
                const int row = row0 + 8 * (i >> 2) + (i & 3);
                if (row < m && exc_segment(need, thr) == j) {
                    if (idx < cap) list[(int64_t)j * cap + idx] = make_int4(row, col, (int)need, 0);
                    ++idx;
                }
            }
        }
    }
}

// The fix-up: one wave per listed cell of segments 0 .. last (every cell
// whose need exceeds the chosen width).  The dot product of the cell's row
// of op(A) and column of op(B) is compensated
// (Ogita, Rump and Oishi's Dot2: each product split exactly into its
// rounded value and error by an FMA, each sum by TwoSum, the errors summed
// apart), per lane over every 64th position, then over the lanes by the same
// steps; the result is within about one rounding of the exact value.
__device__ inline void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double z = s - a;
    e = (a - (s - z)) + (b - z);
}

__global__ void __launch_bounds__(kThreads)
exception_fixup_kernel(const int4 *__restrict__ list, const StatusBlock *st, uint32_t cap,
                       int last, int k, const double *__restrict__ Za, int64_t lda, int axa,
                       const double *__restrict__ Zb, int64_t ldb, int axb,
                       double *__restrict__ C, int64_t ldc) {
    const int lane = threadIdx.x & 63;
    const uint32_t nw = gridDim.x * (kThreads / 64);
    // entries of segments 0 .. last, numbered one after the other
    uint32_t seg_n[kExcThresholds], total = 0;
#pragma unroll
    for (int j = 0; j < kExcThresholds; ++j) {
        seg_n[j] = j <= last ? min(st->exc_seg[j], cap) : 0u;
        total += seg_n[j];
    }
    for (uint32_t e = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); e < total; e += nw) {
        uint32_t j = 0, i = e;
#pragma unroll
        for (int jj = 0; jj < kExcThresholds - 1; ++jj)
            if (j == (uint32_t)jj && i >= seg_n[jj]) {
                i -= seg_n[jj];
                j = jj + 1;
            }
        const int4 cell = list[(int64_t)j * cap + i];
        const int64_t row = cell.x, col = cell.y;
        double sum = 0.0, err = 0.0;
        for (int t = lane; t < k; t += 64) {
            const double x = axa == 0 ? Za[row * lda + t] : Za[(int64_t)t * lda + row];
            const double y = axb == 0 ? Zb[col * ldb + t] : Zb[(int64_t)t * ldb + col];
            const double p = x * y;
            const double pe = fma(x, y, -p);
            double se;
            two_sum(sum, p, sum, se);
            err += pe + se;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double s2 = __shfl_xor(sum, off), e2 = __shfl_xor(err, off);
            double se;
            two_sum(sum, s2, sum, se);
            err += e2 + se;
        }
        if (lane == 0) C[row * ldc + col] = sum + err;
    }
}

}  // namespace

hipError_t launch_need_scan(const uint8_t *plane, int m, int n, ExcThresholds thr, int4 *list,
                            uint32_t cap, StatusBlock *st, hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    const int64_t chunks = (int64_t)((m + 31) / 32) * n * 2;
    const int64_t blocks = std::min<int64_t>((chunks + kThreads - 1) / kThreads, 4096);
    need_scan_kernel<<<(unsigned)blocks, kThreads, 0, s>>>(plane, m, n, thr, list, cap, st);
    return hipGetLastError();
}

hipError_t launch_exception_fixup(const int4 *list, const StatusBlock *st, uint32_t cap, int last,
                                  int k, const double *Za, int64_t lda, int axa, const double *Zb,
                                  int64_t ldb, int axb, double *C, int64_t ldc, hipStream_t s) {
    if (cap == 0 || last < 0 || last >= kExcThresholds) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)std::min<uint32_t>(((last + 1) * cap + 3) / 4, 1024u);
    exception_fixup_kernel<<<blocks, kThreads, 0, s>>>(list, st, cap, last, k, Za, lda, axa, Zb,
                                                       ldb, axb, C, ldc);
    return hipGetLastError();
}

hipError_t launch_mag_plane(const double *Z, int rows, int cols, int64_t ld, int axis,
                            const unsigned long long *maxbits, const double *sums, double *shat,
                            unsigned long long *umax, int8_t *out, int lines_pad, int len_pad,
                            hipStream_t s) {
    if (rows < 1 || cols < 1 || lines_pad % 64 || len_pad % 64) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(len_pad / 64), (unsigned)(lines_pad / 64));
    if (axis == 0)
        mag_rows_kernel<<<grid, kThreads, 0, s>>>(Z, rows, cols, ld, maxbits, sums, shat, umax,
                                                  out, lines_pad);
    else
        mag_cols_kernel<<<dim3(grid.y, grid.x), kThreads, 0, s>>>(Z, rows, cols, ld, maxbits,
                                                                  sums, col_sum_parts(rows),
                                                                  shat, umax, out, lines_pad);
    return hipGetLastError();
}

hipError_t launch_certify(int m, int n, int k, const int8_t *qa, int a_lines_pad,
                          const int8_t *qb, int b_lines_pad, int len_pad, const CertArgs &ca,
                          bool digits, hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    if (!crt_planes_ok(m, n, k, a_lines_pad, b_lines_pad, len_pad)) return hipErrorInvalidValue;
    TraceScope ts(TCU_KERNEL_CERTIFY, m, n, k, 1, 2.0 * m * n * (double)k, s);
    const bool wide = crt_tile_cols(n) == CrtCfgWide::BN;
    if (digits)
        return wide ? gemm_crt_single<CrtCfgWide, kEpiCertifyDigits>(
                          m, n, k, qa, a_lines_pad, qb, b_lines_pad, len_pad, ca, nullptr, 0, s)
                    : gemm_crt_single<CrtCfg, kEpiCertifyDigits>(
                          m, n, k, qa, a_lines_pad, qb, b_lines_pad, len_pad, ca, nullptr, 0, s);
    return wide ? gemm_crt_single<CrtCfgWide, kEpiCertify>(m, n, k, qa, a_lines_pad, qb,
                                                            b_lines_pad, len_pad, ca, nullptr, 0, s)
                : gemm_crt_single<CrtCfg, kEpiCertify>(m, n, k, qa, a_lines_pad, qb, b_lines_pad,
                                                        len_pad, ca, nullptr, 0, s);
}

// A 1 at (line = group, position = key) of every in-range record of R in its
// 0/1 plane (zeroed first); plain byte stores (unique cells).  Skipped
// records were counted by the value encoding already.
__global__ void __launch_bounds__(kThreads)
count_plane_kernel(int64_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ key,
                   int lines, int len, int8_t *__restrict__ plane, int lines_pad) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int g = grp[i], k = key[i];
    if ((unsigned)g < (unsigned)lines && (unsigned)k < (unsigned)len)
        plane[res_offset(g, k, lines_pad)] = 1;
}

hipError_t launch_count_planes(const tcu_relation &R, int lines, int len, int8_t *plane,
                               int lines_pad, int len_pad, hipStream_t s) {
    if (lines_pad < lines || len_pad < len || lines_pad % 64 || len_pad % 64)
        return hipErrorInvalidValue;
    // zeroed by a kernel, not a memset node (the call may be captured)
    hipError_t e = launch_zero_f64(reinterpret_cast<double *>(plane),
                                   (size_t)lines_pad * len_pad / 8, s);
    if (e != hipSuccess || R.n == 0) return e;
    count_plane_kernel<<<(unsigned)((R.n + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        R.n, R.group, R.key, lines, len, plane, lines_pad);
    return hipGetLastError();
}

hipError_t launch_count_product(int m, int n, int k, const int8_t *qa, int a_lines_pad,
                                const int8_t *qb, int b_lines_pad, int len_pad, int32_t *count,
                                int64_t ldc, hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    if (!crt_planes_ok(m, n, k, a_lines_pad, b_lines_pad, len_pad)) return hipErrorInvalidValue;
    TraceScope ts(TCU_KERNEL_COUNT, m, n, k, 1, 2.0 * m * n * (double)k, s);
    const CertArgs none{};
    return crt_tile_cols(n) == CrtCfgWide::BN
               ? gemm_crt_single<CrtCfgWide, kEpiCount>(m, n, k, qa, a_lines_pad, qb, b_lines_pad,
                                                         len_pad, none, count, ldc, s)
               : gemm_crt_single<CrtCfg, kEpiCount>(m, n, k, qa, a_lines_pad, qb, b_lines_pad,
                                                     len_pad, none, count, ldc, s);
}

}  // namespace tcu
