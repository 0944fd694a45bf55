// gemm_split.hip -- step a2 in the mixed-precision form: the contraction
// C = X * Y of TCUDB Section 3.3 from 7-bit digit slices on the narrow
// matrix cores, exact integer partial sums, FP64 combination.
//
// With X[g,k] = 2^e_g sum_p dX_p[g,k] 2^(-7p) and Y[k,h] = 2^f_h sum_q
// dY_q[k,h] 2^(-7q) (split.hip), the kernel evaluates
//   C[g,h] = 2^(e_g + f_h) * sum_{t=2}^{S+1} 2^(-7t) * sum_{p+q=t} sum_k dX_p dY_q
// i.e. all digit pairs on the first S anti-diagonals, each later diagonal a
// correction of the previous ones 2^-7 times smaller.  Each inner sum of
// digit products is an integer: every product is below 2^14 in magnitude,
// so a diagonal with D pairs accumulated over L values of k stays exact in
// the accumulator as long as D * L * 127^2 fits (2^31 for int32, 2^24 for
// FP32).  BF16 accumulators are flushed into an FP64 sum held in registers
// every 128 k (S = 7); int8 accumulators stay exact over 16384 k, so a
// longer contraction is cut into launches of that length that add into C.
//
// Matrix-core instructions (gfx950), lane layouts measured on the device:
//   v_mfma_i32_32x32x32_i8 / v_mfma_f32_32x32x16_bf16: A lane l holds row
//   l%32, k in [KSTEP/2 * (l/32), +KSTEP/2); B lane l holds column l%32, the
//   same k range; D lane l item i is row 8*(i/4) + 4*(l/32) + i%4, col l%32.
// Both consume 16 bytes per lane per operand per k-step (KSTEP = 32 int8
// digits or 16 BF16 digits).
//
// Tiling: 4 waves in a 2 x 2 grid; a wave owns 32 x 64 outputs (int8: two
// 32 x 32 blocks, workgroup 64 x 128) or 32 x 32 (BF16, which also holds the
// FP64 sum; workgroup 64 x 64).  One pipeline stage is one k-step of all S
// slices of both operands, moved global -> LDS by direct-to-LDS loads (no
// register staging) into three rotating buffers, so the loads of a k-step
// are issued two k-steps before it is multiplied.  Each wave holds one
// accumulator per diagonal and block (S * WNB * 16 registers) and reads each
// slice's fragment once per k-step, so the S(S+1)/2 digit products reuse
// registers instead of LDS.
#include <type_traits>

#include "internal.h"

namespace tcu {
namespace {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64;  // workgroup rows (2 waves of 32)
constexpr int GROUP_M = 8;
constexpr int NUM_XCD = 8;

template <typename T> struct Mfma;
template <> struct Mfma<int8_t> {
    using acc_t = i16v;
    static constexpr long kExactLimit = 2147483647L;  // int32
    static constexpr int kWNB = 1;                    // 32 x 32 blocks per wave along n
    static constexpr int kWavesN = 4;                 // waves along n (8 per workgroup)
    static constexpr bool kSum = false;               // one exact chunk per launch
    __device__ static inline acc_t step(i4 a, i4 b, acc_t c) {
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<uint16_t> {
    using acc_t = f16v;
    static constexpr long kExactLimit = 16777216L;  // integers exact in FP32
    static constexpr int kWNB = 1;
    static constexpr int kWavesN = 2;
    static constexpr bool kSum = true;              // FP64 sum over short exact chunks
    __device__ static inline acc_t step(i4 a, i4 b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, a),
                                                       __builtin_bit_cast(bf8, b), c, 0, 0, 0);
    }
};

// k-steps per exact chunk: the largest power of two with S * L * 127^2 exact
template <typename T>
inline int flush_steps(int S) {
    const int kstep = 32 / (int)sizeof(T);
    const long L = Mfma<T>::kExactLimit / ((long)S * 16129L) / kstep;
    int f = 1;
    while ((long)f * 2 <= L && f < (1 << 20)) f *= 2;
    return f;
}

__device__ inline void tile_coords(int tiles_m, int tiles_n, int &tm, int &tn) {
    const int nt = tiles_m * tiles_n;
    const int wg = blockIdx.x;
    const int per = nt / NUM_XCD;
    const int full = per * NUM_XCD;
    const int logical = wg < full ? (wg % NUM_XCD) * per + wg / NUM_XCD : wg;
    const int group = GROUP_M * tiles_n;
    const int first_m = (logical / group) * GROUP_M;
    const int gm = min(tiles_m - first_m, GROUP_M);
    const int in_group = logical % group;
    tm = first_m + in_group % gm;
    tn = in_group / gm;
}

// One pipeline stage = one k-step of all S slices of both operands:
// X planes [S][2 halves][BM rows][16 B], then Y planes [S][2][BN rows][16 B].
// Each (slice, half, 64-row block) plane is one 1 KB run in global memory
// (split.hip's layout) and one wave instruction, global_load_lds_dwordx4,
// moves it straight into LDS: lane l's 16 bytes land at plane base + 16 l.
template <int S, int BN, int NW>
struct Stage {
    static constexpr int xi = S * 2;                // X planes (BM = 64 rows)
    static constexpr int yi = S * 2 * (BN / 64);    // Y planes
    static constexpr int planes = xi + yi;
    static constexpr int per_wave = (planes + NW - 1) / NW;
    static constexpr int chunks = planes * 64 + 64; // + one scratch plane
    static constexpr int x_chunks = xi * 64;
};

constexpr int NSTAGE = 3;  // LDS buffers: loads run two k-steps ahead of the fragment reads

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding:
// vmcnt bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]).
template <int V>
__device__ inline void wait_vmcnt() {
    static_assert(V >= 0 && V < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((V & 15) | ((V >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier without the memory fence __syncthreads() implies: that
// fence makes the compiler wait for every outstanding load, including the
// direct-to-LDS loads of later k-steps.  Completion of this wave's LDS-bound
// loads is waited for explicitly (wait_vmcnt), LDS reads complete before
// their MFMAs use them, and the "memory" clobber keeps the compiler from
// moving LDS accesses across the barrier.
__device__ inline void barrier_no_fence() { asm volatile("s_barrier" ::: "memory"); }

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void global_cvoid;

// While the matrix cores are kept busy, vector-ALU instructions of every
// wave on the SIMD get few issue slots, so the main loop does its address
// arithmetic on the scalar unit: each direct-to-LDS load is a uniform SGPR
// base plus the lane's fixed byte offset (the SADDR form), with its LDS
// address in M0.
__device__ inline void load_lds16(const char *sbase, unsigned voff, unsigned lds_addr) {
    asm volatile("global_load_lds_dwordx4 %0, %1" : : "v"(voff), "s"(sbase), "{m0}"(lds_addr)
                 : "memory");
}

// A uniform address computed on the vector ALU (64-bit products are) moved to
// scalar registers; the builtin returns int, so widen through uint32_t.
__device__ inline const char *to_sgpr(const char *p) {
    const uint64_t u = (uint64_t)(uintptr_t)p;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((unsigned)u);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (const char *)(uintptr_t)(lo | (hi << 32));
}

// This wave's share of every stage's loads.  Plane q (wave-uniform) goes to
// wave q % NW; waves with fewer real planes load a valid dummy run into the
// scratch plane, so every wave issues exactly per_wave instructions and its
// vmcnt bookkeeping is a constant.  Load j of k-step kb reads
// src[j] + kb * step[j] (+ the lane's 16 bytes) into stage offset dst[j].
template <int S, int BN, int NW>
struct WaveLoads {
    using St = Stage<S, BN, NW>;
    const char *src[St::per_wave];
    int64_t step[St::per_wave];
    unsigned dst[St::per_wave];
};

template <int S, int BN, int NW>
__device__ inline WaveLoads<S, BN, NW> wave_loads(int wave, int nblk, const char *xs,
                                                  int x_lines_pad, int m0, const char *ys,
                                                  int y_lines_pad, int n0) {
    using St = Stage<S, BN, NW>;
    WaveLoads<S, BN, NW> L;
#pragma unroll
    for (int j = 0; j < St::per_wave; ++j) {
        const int q = wave + NW * j;
        const char *src;
        if (q < St::xi) {
            const int p = q >> 1, h = q & 1;
            src = xs + ((((int64_t)p * nblk) * 2 + h) * x_lines_pad + m0) * 16;
            L.step[j] = (int64_t)2 * x_lines_pad * 16;
            L.dst[j] = (unsigned)q * 64u * 16u;
        } else if (q < St::planes) {
            const int qq = q - St::xi;
            const int rb = qq % (BN / 64), ph = qq / (BN / 64);
            const int p = ph >> 1, h = ph & 1;
            src = ys + ((((int64_t)p * nblk) * 2 + h) * y_lines_pad + n0 + rb * 64) * 16;
            L.step[j] = (int64_t)2 * y_lines_pad * 16;
            L.dst[j] = (unsigned)q * 64u * 16u;
        } else {
            src = xs;
            L.step[j] = 0;
            L.dst[j] = (unsigned)St::planes * 64u * 16u;
        }
        L.src[j] = to_sgpr(src);
    }
    return L;
}

template <int S, int BN, int NW>
__device__ inline void issue_stage(const WaveLoads<S, BN, NW> &L, int kb, unsigned buf_addr,
                                   unsigned voff) {
#pragma unroll
    for (int j = 0; j < Stage<S, BN, NW>::per_wave; ++j)
        load_lds16(L.src[j] + (int64_t)kb * L.step[j], voff, buf_addr + L.dst[j]);
}

// Digit products of slices p in [P0, P1) with every q on the kept diagonals.
template <typename T, int S, int WNB, int P0, int P1>
__device__ inline void mfma_range(const i4 (&fx)[S], const i4 (&fy)[S][WNB],
                                  typename Mfma<T>::acc_t (&acc)[S][WNB]) {
#pragma unroll
    for (int p = P0; p < P1; ++p)
#pragma unroll
        for (int q = 0; q + p < S; ++q)
#pragma unroll
            for (int b = 0; b < WNB; ++b) acc[p + q][b] = Mfma<T>::step(fx[p], fy[q][b], acc[p + q][b]);
}

// k-steps [kb0, kb1) of the product; accumulate != 0 adds to C.
//
// Software pipeline, per k-step kb (fragments of kb already in registers):
//   1. the MFMAs of the first slices of X;
//   2. wait for this wave's loads of k-step kb+1, barrier (every wave's
//      loads of kb+1 have landed, and every wave has consumed its fragments
//      of kb, so kb's LDS buffer is free);
//   3. issue the direct-to-LDS loads of k-step kb+3 into that buffer;
//   4. read the fragments of kb+1 from LDS while
//   5. the MFMAs of the remaining slices of X run.
// The LDS read latency and the barrier then overlap matrix-core work, with
// one wave per SIMD.  Fragments alternate between two register sets (the
// loop is unrolled by two), global loads run two k-steps ahead.
template <typename T>
constexpr int split_threads() { return 64 * 2 * Mfma<T>::kWavesN; }

template <typename T, int S>
__global__ void __launch_bounds__(split_threads<T>())
gemm_split_kernel(int m, int n, int nblk, int kb0, int kb1, int flush, int accumulate,
                  const char *__restrict__ xs, int x_lines_pad, const char *__restrict__ ys,
                  int y_lines_pad, const int *__restrict__ ex, const int *__restrict__ ey,
                  double *__restrict__ C, int64_t ldc) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int WNB = M::kWNB;
    constexpr int NW = 2 * M::kWavesN;
    constexpr int BN = 32 * WNB * M::kWavesN;
    constexpr int PSPLIT = (S + 1) / 3;  // slices of X multiplied before the barrier
    using St = Stage<S, BN, NW>;
    __shared__ __attribute__((aligned(16))) i4 lds[NSTAGE][St::chunks];

    const int tiles_m = (m + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    // the wave index is uniform across the wave: in a scalar register, the
    // plane selection of the loads is scalar
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int l32 = lane & 31, half = lane >> 5;
    const unsigned voff = (unsigned)lane * 16u;
    const unsigned lds_addr = (unsigned)(uintptr_t)&lds[0][0];
    const WaveLoads<S, BN, NW> L =
        wave_loads<S, BN, NW>(wave, nblk, xs, x_lines_pad, m0, ys, y_lines_pad, n0);
    // this lane's fragment bases; buffer, slice and block offsets are constants
    const i4 *lx = &lds[0][0] + half * BM + wm * 32 + l32;
    const i4 *ly = &lds[0][0] + St::x_chunks + half * BN + wn * 32 * WNB + l32;

    acc_t acc[S][WNB];
    double sum[M::kSum ? WNB : 1][M::kSum ? 16 : 1];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int b = 0; b < WNB; ++b) acc[d][b] = acc_t{};
    if constexpr (M::kSum) {
#pragma unroll
        for (int b = 0; b < WNB; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) sum[b][i] = 0.0;
    }

    auto flush_sum = [&]() {
        if constexpr (M::kSum) {
#pragma unroll
            for (int d = 0; d < S; ++d)
#pragma unroll
                for (int b = 0; b < WNB; ++b) {
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        sum[b][i] += ldexp((double)acc[d][b][i], -7 * (d + 2));
                    acc[d][b] = acc_t{};
                }
        }
    };

    i4 f0x[S], f0y[S][WNB], f1x[S], f1y[S][WNB];
    // fragments of the k-step in LDS buffer B
    auto read = [&](auto Bc, i4 (&fx)[S], i4 (&fy)[S][WNB]) {
        constexpr int B = decltype(Bc)::value;
#pragma unroll
        for (int p = 0; p < S; ++p) {
            fx[p] = lx[B * St::chunks + p * 2 * BM];
#pragma unroll
            for (int b = 0; b < WNB; ++b) fy[p][b] = ly[B * St::chunks + p * 2 * BN + b * 32];
        }
    };

    // one k-step; IT3 = (kb - kb0) mod 3 is its LDS buffer, REG = (kb - kb0)
    // mod 2 its fragment register set (the other set receives the next
    // k-step's fragments)
    auto kstep = [&](auto IT3c, auto REGc, int kb) {
        constexpr int IT3 = decltype(IT3c)::value, REG = decltype(REGc)::value;
        i4(&fcx)[S] = REG == 0 ? f0x : f1x;
        i4(&fcy)[S][WNB] = REG == 0 ? f0y : f1y;
        i4(&fnx)[S] = REG == 0 ? f1x : f0x;
        i4(&fny)[S][WNB] = REG == 0 ? f1y : f0y;
        mfma_range<T, S, WNB, 0, PSPLIT>(fcx, fcy, acc);
        __builtin_amdgcn_sched_barrier(0);
        if (kb + 1 < kb1) {
            if (kb + 2 < kb1) wait_vmcnt<St::per_wave>();
            else wait_vmcnt<0>();
            barrier_no_fence();
            // kb's buffer is free: every wave has read its fragments
            if (kb + 3 < kb1)
                issue_stage<S, BN, NW>(L, kb + 3, lds_addr + (unsigned)IT3 * St::chunks * 16u, voff);
            read(std::integral_constant<int, (IT3 + 1) % NSTAGE>{}, fnx, fny);
        }
        __builtin_amdgcn_sched_barrier(0);
        mfma_range<T, S, WNB, PSPLIT, S>(fcx, fcy, acc);
        if constexpr (M::kSum) {
            if ((kb - kb0 + 1) % flush == 0 || kb + 1 == kb1) flush_sum();
        }
    };

    // prologue: k-steps kb0 .. kb0 + 2 in flight, fragments of kb0 read
#pragma unroll
    for (int st = 0; st < NSTAGE; ++st)
        if (kb0 + st < kb1)
            issue_stage<S, BN, NW>(L, kb0 + st, lds_addr + (unsigned)st * St::chunks * 16u, voff);
    const int issued = kb1 - kb0 < NSTAGE ? kb1 - kb0 : NSTAGE;
    if (issued == 3) wait_vmcnt<2 * St::per_wave>();
    else if (issued == 2) wait_vmcnt<St::per_wave>();
    else wait_vmcnt<0>();
    barrier_no_fence();
    read(std::integral_constant<int, 0>{}, f0x, f0y);

    // unrolled by 6 so the LDS buffer (period 3) and the register set
    // (period 2) of every k-step are compile-time constants
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    for (int kb = kb0; kb < kb1; kb += 6) {
        kstep(I0{}, I0{}, kb);
        if (kb + 1 < kb1) kstep(I1{}, I1{}, kb + 1);
        if (kb + 2 < kb1) kstep(I2{}, I0{}, kb + 2);
        if (kb + 3 < kb1) kstep(I0{}, I1{}, kb + 3);
        if (kb + 4 < kb1) kstep(I1{}, I0{}, kb + 4);
        if (kb + 5 < kb1) kstep(I2{}, I1{}, kb + 5);
    }

    // epilogue: C (+)= 2^(e_g + f_h) * sum_t 2^(-7t) S_t
#pragma unroll
    for (int b = 0; b < WNB; ++b) {
        const int col = n0 + wn * 32 * WNB + b * 32 + l32;
        if (col >= n) continue;
        const int fcol = ey[col];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = m0 + wm * 32 + 8 * (i >> 2) + 4 * half + (i & 3);
            if (row >= m) continue;
            double v;
            if constexpr (M::kSum) {
                v = sum[b][i];
            } else {
                v = 0.0;
#pragma unroll
                for (int d = S - 1; d >= 0; --d) v += ldexp((double)acc[d][b][i], -7 * (d + 2));
            }
            v = ldexp(v, ex[row] + fcol);
            double *dst = C + (int64_t)row * ldc + col;
            *dst = accumulate ? *dst + v : v;
        }
    }
}

template <typename T, int S>
hipError_t launch_s(int m, int n, int nblk, const void *xs, int x_lines_pad, const void *ys,
                    int y_lines_pad, const int *ex, const int *ey, double *C, int64_t ldc,
                    hipStream_t s) {
    constexpr int BN = 32 * Mfma<T>::kWNB * Mfma<T>::kWavesN;
    const int tiles = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    const int flush = flush_steps<T>(S);
    // int8: one launch per exact chunk (no FP64 sum held in registers);
    // BF16: one launch, flushing into the FP64 sum every `flush` k-steps
    const int chunk = Mfma<T>::kSum ? nblk : flush;
    for (int kb0 = 0; kb0 < nblk; kb0 += chunk) {
        const int kb1 = kb0 + chunk < nblk ? kb0 + chunk : nblk;
        const int kstep = 32 / (int)sizeof(T);
        const double kk = (double)(kb1 - kb0) * kstep;
        TraceScope ts(TCU_KERNEL_GEMM_SPLIT, m, n, (int)kk, S, S * (S + 1) / 2 * 2.0 * m * n * kk,
                      s);
        gemm_split_kernel<T, S><<<tiles, split_threads<T>(), 0, s>>>(
            m, n, nblk, kb0, kb1, flush, kb0 > 0, static_cast<const char *>(xs), x_lines_pad,
            static_cast<const char *>(ys), y_lines_pad, ex, ey, C, ldc);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_t(int m, int n, int nblk, int S, const void *xs, int x_lines_pad,
                    const void *ys, int y_lines_pad, const int *ex, const int *ey, double *C,
                    int64_t ldc, hipStream_t s) {
    switch (S) {
#define TCU_GS_CASE(v) \
    case v: return launch_s<T, v>(m, n, nblk, xs, x_lines_pad, ys, y_lines_pad, ex, ey, C, ldc, s);
        TCU_GS_CASE(1) TCU_GS_CASE(2) TCU_GS_CASE(3) TCU_GS_CASE(4)
        TCU_GS_CASE(5) TCU_GS_CASE(6) TCU_GS_CASE(7) TCU_GS_CASE(8)
#undef TCU_GS_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace

int split_chunk_steps(int S, int digit_bf16) {
    return digit_bf16 ? flush_steps<uint16_t>(S) : flush_steps<int8_t>(S);
}

hipError_t launch_gemm_split(int m, int n, int k, int S, int digit_bf16, const void *xs,
                             int x_lines_pad, const void *ys, int y_lines_pad, int len_pad,
                             const int *ex, const int *ey, double *C, int64_t ldc,
                             hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    if (x_lines_pad % 128 || y_lines_pad % 128 || len_pad % 64 || len_pad < k)
        return hipErrorInvalidValue;
    if (x_lines_pad < m || y_lines_pad < n) return hipErrorInvalidValue;
    const int kstep = digit_bf16 ? 16 : 32;
    const int nblk = len_pad / kstep;
    if (nblk == 0) return hipErrorInvalidValue;
    if (digit_bf16)
        return launch_t<uint16_t>(m, n, nblk, S, xs, x_lines_pad, ys, y_lines_pad, ex, ey, C,
                                  ldc, s);
    return launch_t<int8_t>(m, n, nblk, S, xs, x_lines_pad, ys, y_lines_pad, ex, ey, C, ldc, s);
}

}  // namespace tcu
