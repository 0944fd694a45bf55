// split.hip -- step a0 of the mixed-precision form: per-line statistics and
// the fixed-point slicing of an FP64 encoding into narrow integer digits.
//
// TCUDB's feasibility test (Section 4.2.1) reads per-column min/max metadata
// to pick the narrowest matrix-unit type that still gives acceptable results,
// or refuses.  The mixed form generalises it: every line (row of X, column of
// Y) gets a power-of-two scale from its largest magnitude, and the scaled
// values are cut into S digits of 7 bits that the matrix units multiply
// exactly:
//   mx   = max |z| over the line,  e = exponent with 2^(e-1) <= mx < 2^e
//          (e = 0 for an all-zero line),
//   r_0  = z * 2^-e,  t = r_{p-1} * 2^7,  d_p = trunc(t),  r_p = t - d_p,
// so z = 2^e (sum_p d_p 2^(-7p) + r_S 2^(-7S)) exactly, |d_p| <= 127, and
// every step is exact in FP64 (power-of-two scalings, removal of an
// integer part).  Digits are stored as int8 or as BF16 (|d| <= 127 has at
// most 7 significant bits, exact in BF16).
//
// Output layout, blocked for the split GEMM's loads: the position t along a
// line is cut into k-steps of 32 bytes of digits (KSTEP = 32 int8 or 16 BF16
// digits, one matrix-core k-step), each k-step into two 16-byte halves
// (HALF = KSTEP / 2 digits, the slice of k one lane feeds the matrix core),
// and
//   slices[p][t / KSTEP][(t % KSTEP) / HALF][line][t % HALF]
// so the 16-byte halves of 64 consecutive lines are one contiguous 1 KB run,
// which one wave loads straight into LDS.  Lines are padded with zero digits
// to `lines_pad` (a multiple of 128) and t to `len_pad` (a multiple of 64);
// slice p starts at p * lines_pad * len_pad.
// Lines are rows of the input (no transpose) or its columns (transposed
// through LDS).
//
// Both kernels are HBM-bound: the statistics read 8 B per element, the split
// reads 8 B and writes S * sizeof(digit) B per element.
#include "internal.h"

namespace tcu {
namespace {

constexpr int kThreads = 256;
constexpr int kDigitBits = 7;

__device__ inline unsigned long long abs_bits(double z) {
    return (unsigned long long)__double_as_longlong(fabs(z));
}

// Max |z| and sum of |z| per row: one wave per row.  Each lane adds its
// columns in a fixed order and lane 0 combines the lanes in a fixed order,
// so the sum is the same on every run.
__global__ void __launch_bounds__(kThreads)
row_max_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld,
               unsigned long long *__restrict__ maxbits, double *__restrict__ sums,
               StatusBlock *st) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * (kThreads / 64) + wave;
    if (row >= rows) return;
    const double *z = Z + (int64_t)row * ld;
    // eight independent loads in flight per lane (the loop is latency-bound
    // with one)
    double m[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool bad = false;
    int c = lane;
    for (; c + 7 * 64 < cols; c += 8 * 64) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = z[c + 64 * u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            bad |= !isfinite(v[u]);
            m[u] = fmax(m[u], fabs(v[u]));
            a[u] += fabs(v[u]);
        }
    }
    for (; c < cols; c += 64) {
        const double v = z[c];
        bad |= !isfinite(v);
        m[0] = fmax(m[0], fabs(v));
        a[0] += fabs(v);
    }
    double mx = fmax(fmax(fmax(m[0], m[1]), fmax(m[2], m[3])), fmax(fmax(m[4], m[5]), fmax(m[6], m[7])));
    double sm = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    // lane 0 ends with the same association of the 64 lane sums on every run
    for (int off = 32; off > 0; off >>= 1) sm += __shfl_down(sm, off);
    const unsigned long long anybad = __ballot(bad);
    if (lane == 0) {
        maxbits[row] = abs_bits(mx);
        if (sums != nullptr) sums[row] = sm;
        if (anybad) atomicOr(&st->flags, kFlagNonFinite);
    }
}

// Max |z| and sum of |z| per column: threads own columns, blocks own chunks
// of rows.  The partial maxima meet in an atomic max on the (monotone) bit
// patterns of the non-negative doubles (maxbits must be zero beforehand);
// the partial sums of chunk y go to sums[y * cols + col], and
// col_sum_parts(rows) chunks are later added in order (line_abs_sum), so the
// column sums do not depend on the order in which blocks run.
__global__ void __launch_bounds__(kThreads)
col_max_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld, int chunk,
               unsigned long long *__restrict__ maxbits, double *__restrict__ sums,
               StatusBlock *st) {
    const int col = blockIdx.x * kThreads + threadIdx.x;
    const int r0 = blockIdx.y * chunk;
    const int r1 = min(rows, r0 + chunk);
    double mx = 0.0;
    bool bad = false;
    if (col < cols) {
        // eight independent loads in flight per thread
        double m[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const double *z = Z + col;
        int r = r0;
        int64_t off = (int64_t)r0 * ld;  // element offset of row r (a running sum)
        for (; r + 7 < r1; r += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = z[off + u * ld];
            off += 8 * ld;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                bad |= !isfinite(v[u]);
                m[u] = fmax(m[u], fabs(v[u]));
                a[u] += fabs(v[u]);
            }
        }
        for (; r < r1; ++r, off += ld) {
            const double v = z[off];
            bad |= !isfinite(v);
            m[0] = fmax(m[0], fabs(v));
            a[0] += fabs(v);
        }
        mx = fmax(fmax(fmax(m[0], m[1]), fmax(m[2], m[3])), fmax(fmax(m[4], m[5]), fmax(m[6], m[7])));
        atomicMax(maxbits + col, abs_bits(mx));
        if (sums != nullptr)
            sums[(int64_t)blockIdx.y * cols + col] =
                ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    const unsigned long long anybad = __ballot(bad);
    if (anybad && (threadIdx.x & 63) == 0) atomicOr(&st->flags, kFlagNonFinite);
}

__device__ inline int line_exponent(unsigned long long bits) {
    const double mx = __longlong_as_double((long long)bits);
    int e = 0;
    if (mx > 0.0) frexp(mx, &e);
    return e;
}

template <typename T> __device__ inline T to_digit(double d);
template <> __device__ inline int8_t to_digit<int8_t>(double d) { return (int8_t)(int)d; }
template <> __device__ inline uint16_t to_digit<uint16_t>(double d) {
    // |d| <= 127 is exact in FP32 and its low 16 mantissa bits are zero
    return (uint16_t)(__float_as_uint((float)d) >> 16);
}

// One vector store of 8 digits (8 B of int8 or 16 B of BF16); the slice
// layout keeps every group of 8 aligned.
__device__ inline void store8(int8_t *dst, const int8_t (&d)[8]) {
    uint2 v;
    v.x = (uint32_t)(uint8_t)d[0] | ((uint32_t)(uint8_t)d[1] << 8) |
          ((uint32_t)(uint8_t)d[2] << 16) | ((uint32_t)(uint8_t)d[3] << 24);
    v.y = (uint32_t)(uint8_t)d[4] | ((uint32_t)(uint8_t)d[5] << 8) |
          ((uint32_t)(uint8_t)d[6] << 16) | ((uint32_t)(uint8_t)d[7] << 24);
    *reinterpret_cast<uint2 *>(dst) = v;
}
__device__ inline void store8(uint16_t *dst, const uint16_t (&d)[8]) {
    uint4 v;
    v.x = (uint32_t)d[0] | ((uint32_t)d[1] << 16);
    v.y = (uint32_t)d[2] | ((uint32_t)d[3] << 16);
    v.z = (uint32_t)d[4] | ((uint32_t)d[5] << 16);
    v.w = (uint32_t)d[6] | ((uint32_t)d[7] << 16);
    *reinterpret_cast<uint4 *>(dst) = v;
}

template <typename T>
__device__ inline int64_t slice_offset(int line, int t, int lines_pad) {
    constexpr int kstep = 32 / (int)sizeof(T), half = kstep / 2;
    const int kb = t / kstep, h = (t % kstep) / half;
    return (((int64_t)kb * 2 + h) * lines_pad + line) * half + (t % half);
}

// 16 consecutive digits of one line (positions t0 .. t0 + 15, t0 a multiple
// of 16) at their slice-layout place: one 16-byte store for int8 (one half
// k-step), two for BF16 (the two halves of one k-step).
__device__ inline void store16(int8_t *slice, int line, int t0, int lines_pad,
                               const int8_t (&d)[16]) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        w[q] = (uint32_t)(uint8_t)d[4 * q] | ((uint32_t)(uint8_t)d[4 * q + 1] << 8) |
               ((uint32_t)(uint8_t)d[4 * q + 2] << 16) | ((uint32_t)(uint8_t)d[4 * q + 3] << 24);
    *reinterpret_cast<uint4 *>(slice + slice_offset<int8_t>(line, t0, lines_pad)) =
        make_uint4(w[0], w[1], w[2], w[3]);
}
__device__ inline void store16(uint16_t *slice, int line, int t0, int lines_pad,
                               const uint16_t (&d)[16]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint4 v;
        v.x = (uint32_t)d[8 * h] | ((uint32_t)d[8 * h + 1] << 16);
        v.y = (uint32_t)d[8 * h + 2] | ((uint32_t)d[8 * h + 3] << 16);
        v.z = (uint32_t)d[8 * h + 4] | ((uint32_t)d[8 * h + 5] << 16);
        v.w = (uint32_t)d[8 * h + 6] | ((uint32_t)d[8 * h + 7] << 16);
        *reinterpret_cast<uint4 *>(slice + slice_offset<uint16_t>(line, t0 + 8 * h, lines_pad)) = v;
    }
}

// Lines are rows.  One workgroup per 64 lines x 64 positions (grid: len_pad /
// 64, lines_pad / 64): the tile is read row-contiguously into padded LDS,
// then thread (r, g) = (t % 64, t / 64) takes positions 16 g .. 16 g + 15 of
// line l0 + r, so a wave's stores of one slice are one contiguous run per
// slice-layout plane.  Padding rows and columns get zero digits.
template <typename T, int S>
__global__ void __launch_bounds__(kThreads)
split_rows_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld,
                  const unsigned long long *__restrict__ maxbits, T *__restrict__ out,
                  int lines_pad, int len_pad, int *__restrict__ exps) {
    __shared__ double tile[64][64 + 2];  // [line][position]; the pad spreads lines over banks
    const int p0 = blockIdx.x * 64, l0 = blockIdx.y * 64;
    const int t = threadIdx.x;
    // element offset of this thread's load j, advanced by 4 rows per load
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
    const bool live = line < rows;
    const int e = live ? line_exponent(maxbits[line]) : 0;
    if (live && blockIdx.x == 0 && g == 0) exps[line] = e;
    T dig[S][16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        double z = tile[r][16 * g + j];
        if (!isfinite(z)) z = 0.0;
        double rem = ldexp(z, -e);
#pragma unroll
        for (int p = 0; p < S; ++p) {
            const double tt = ldexp(rem, kDigitBits);
            const double d = trunc(tt);
            dig[p][j] = to_digit<T>(d);
            rem = tt - d;
        }
    }
    const int64_t slice_stride = (int64_t)lines_pad * len_pad;
#pragma unroll
    for (int p = 0; p < S; ++p)
        store16(out + (int64_t)p * slice_stride, line, p0 + 16 * g, lines_pad, dig[p]);
}

// Lines are columns: a block turns a 64 x 64 tile of Z into S tiles of
// digits transposed through LDS, so both the FP64 reads and the digit
// writes are contiguous.  Rows in [rows, out_ld) get zero digits.
constexpr int kTile = 64;

template <typename T, int S>
__global__ void __launch_bounds__(kThreads)
split_cols_kernel(const double *__restrict__ Z, int rows, int cols, int64_t ld,
                  const unsigned long long *__restrict__ maxbits, T *__restrict__ out,
                  int lines_pad, int len_pad, int *__restrict__ exps) {
    __shared__ T tile[S][kTile][kTile + 4];  // [p][col][row]
    const int r0 = blockIdx.x * kTile, c0 = blockIdx.y * kTile;
    const int tc = threadIdx.x & 63, tr = threadIdx.x >> 6;  // 4 row lanes
    const int col = c0 + tc;
    const int e = col < cols ? line_exponent(maxbits[col]) : 0;
    if (blockIdx.x == 0 && tr == 0 && col < cols) exps[col] = e;
    // all sixteen loads first, branch-free (element 0 stands in outside the
    // matrix), so they are in flight together
    double zv[kTile / 4];
    int64_t off = (int64_t)(r0 + tr) * ld + col;  // advanced by 4 rows per load
#pragma unroll
    for (int u = 0; u < kTile / 4; ++u) {
        const bool in = r0 + tr + 4 * u < rows && col < cols;
        const double v = Z[in ? off : 0];
        zv[u] = in ? v : 0.0;
        off += 4 * ld;
    }
#pragma unroll
    for (int u = 0; u < kTile / 4; ++u) {
        const int rr = tr + 4 * u;
        double z = zv[u];
        if (!isfinite(z)) z = 0.0;
        double r = ldexp(z, -e);
#pragma unroll
        for (int p = 0; p < S; ++p) {
            const double t = ldexp(r, kDigitBits);
            const double d = trunc(t);
            tile[p][tc][rr] = to_digit<T>(d);
            r = t - d;
        }
    }
    __syncthreads();
    // write: thread -> (column, 16 consecutive rows) of each slice, as two
    // groups of 8 rows (each group lies inside one 16-byte half)
    const int wc = threadIdx.x >> 2, wr = (threadIdx.x & 3) * 16;
    const int ocol = c0 + wc;
    const int64_t slice_stride = (int64_t)lines_pad * len_pad;
#pragma unroll
    for (int p = 0; p < S; ++p) {
        T *base = out + (int64_t)p * slice_stride;
        T v0[8], v1[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) { v0[j] = tile[p][wc][wr + j]; v1[j] = tile[p][wc][wr + 8 + j]; }
        store8(base + slice_offset<T>(ocol, r0 + wr, lines_pad), v0);
        store8(base + slice_offset<T>(ocol, r0 + wr + 8, lines_pad), v1);
    }
}

template <typename T, int S>
hipError_t launch_split_s(const double *Z, int rows, int cols, int64_t ld, int axis,
                          const unsigned long long *maxbits, T *out, int lines_pad, int len_pad,
                          int *exps, hipStream_t s) {
    if (axis == 0) {
        dim3 grid(len_pad / 64, lines_pad / 64);
        split_rows_kernel<T, S><<<grid, kThreads, 0, s>>>(Z, rows, cols, ld, maxbits, out,
                                                          lines_pad, len_pad, exps);
    } else {
        dim3 grid(len_pad / kTile, lines_pad / kTile);
        split_cols_kernel<T, S><<<grid, kThreads, 0, s>>>(Z, rows, cols, ld, maxbits, out,
                                                          lines_pad, len_pad, exps);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_split_t(const double *Z, int rows, int cols, int64_t ld, int axis,
                          const unsigned long long *maxbits, int S, T *out, int lines_pad,
                          int len_pad, int *exps, hipStream_t s) {
    switch (S) {
#define TCU_SPLIT_CASE(n) \
    case n: return launch_split_s<T, n>(Z, rows, cols, ld, axis, maxbits, out, lines_pad, len_pad, exps, s);
        TCU_SPLIT_CASE(1) TCU_SPLIT_CASE(2) TCU_SPLIT_CASE(3) TCU_SPLIT_CASE(4)
        TCU_SPLIT_CASE(5) TCU_SPLIT_CASE(6) TCU_SPLIT_CASE(7) TCU_SPLIT_CASE(8)
#undef TCU_SPLIT_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace

int col_sum_parts(int rows) { return (rows + col_sum_chunk(rows) - 1) / col_sum_chunk(rows); }

int col_sum_chunk(int rows) {
    // at most kColParts chunks, at least 64 rows each, a multiple of 8 rows
    const int c = (rows + kColParts - 1) / kColParts;
    return c < 64 ? 64 : (c + 7) / 8 * 8;
}

hipError_t launch_line_max(const double *Z, int rows, int cols, int64_t ld, int axis,
                           unsigned long long *maxbits, double *sums, StatusBlock *st,
                           hipStream_t s) {
    if (rows == 0 || cols == 0) return hipSuccess;
    if (axis == 0) {
        const unsigned grid = (unsigned)((rows + 3) / 4);
        row_max_kernel<<<grid, kThreads, 0, s>>>(Z, rows, cols, ld, maxbits, sums, st);
    } else {
        // zero the maxima with a kernel (the bit pattern of +0.0 is all zeros)
        hipError_t e = launch_zero_f64(reinterpret_cast<double *>(maxbits), (size_t)cols, s);
        if (e != hipSuccess) return e;
        const int chunk = col_sum_chunk(rows);
        dim3 grid((cols + kThreads - 1) / kThreads, (rows + chunk - 1) / chunk);
        col_max_kernel<<<grid, kThreads, 0, s>>>(Z, rows, cols, ld, chunk, maxbits, sums, st);
    }
    return hipGetLastError();
}

hipError_t launch_split(const double *Z, int rows, int cols, int64_t ld, int axis,
                        const unsigned long long *maxbits, int S, int digit_bf16, void *out,
                        int lines_pad, int len_pad, int *exps, hipStream_t s) {
    // the row kernel reads element 0 in place of positions outside the matrix
    if (rows < 1 || cols < 1 || lines_pad % 128 != 0 || len_pad % 64 != 0)
        return hipErrorInvalidValue;
    if (digit_bf16)
        return launch_split_t<uint16_t>(Z, rows, cols, ld, axis, maxbits, S,
                                        static_cast<uint16_t *>(out), lines_pad, len_pad, exps,
                                        s);
    return launch_split_t<int8_t>(Z, rows, cols, ld, axis, maxbits, S,
                                  static_cast<int8_t *>(out), lines_pad, len_pad, exps, s);
}

}  // namespace tcu
