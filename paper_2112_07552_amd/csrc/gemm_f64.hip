// gemm_f64.hip -- step a2 (the contraction C = X * Y of TCUDB Section 3.3)
// and the two products of the adjoint, in FP64 on the CDNA4 matrix cores.
//
// C (m x n) = op(A) (m x k) * op(B) (k x n), all FP64; C overwritten, or
// (accumulate) C += op(A) op(B).
//
// Design (gfx950):
//  * v_mfma_f64_16x16x4_f64: one wave multiplies a 16x4 by a 4x16 block;
//    A lane holds A[lane%16][lane/16], B lane holds B[lane/16][lane%16], the
//    accumulator lane holds D[lane/16 + 4*i][lane%16], i = 0..3 (measured on
//    gfx950: rows interleave with stride 4 across the lane groups).
//  * Workgroup tile 128 x 128, 4 waves in a 2 x 2 grid, each wave owning a
//    64 x 64 block (4 x 4 MFMA blocks, 64 FP64 accumulators per lane).
//  * K advances in stages of 16 through double-buffered LDS; global loads of
//    stage s+1 are issued before the MFMAs of stage s and written to the other
//    buffer afterwards, so one barrier per stage suffices.
//  * Inside a stage, lane group j = lane/16 at k-step t (0..3) contracts
//    k = 4j + t (any bijection of the 16 k values is a valid contraction
//    order as long as A and B use the same one).  Fragments are read from LDS
//    one k-step at a time, which keeps the kernel within 128 VGPRs + 128
//    AGPRs, so two workgroups (two waves per SIMD) share a CU and cover each
//    other's barrier and load stalls.
//  * Operands whose contraction index is contiguous in memory are staged as
//    [outer][16 + 2] in LDS, the others as [16][128 + 2]; the pads spread rows
//    over the LDS banks.  Global loads are 16-byte vectors when the leading
//    dimension and base address allow, 8-byte guarded loads otherwise.
//  * Tiles are numbered so that each of the 8 XCDs (workgroup w runs on XCD
//    w mod 8) owns a contiguous run of tiles, grouped 8 tile-rows deep, so
//    the A and B panels a run needs stay in that XCD's L2.
//  * Whole-tile launches (the common case: m, n >= 128, k >= 16, 16-byte
//    aligned operands; edge tiles are moved back inside the matrix and a
//    partial last stage of k is added by a second, guarded launch) run a
//    main loop whose address arithmetic is all scalar (see the whole-tile
//    path below): busy matrix cores leave vector-ALU instructions few issue
//    slots.
#include <algorithm>

#include "internal.h"

namespace tcu {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int THREADS = 256;
constexpr int WM = 64, WN = 64;
constexpr int FM = WM / 16, FN = WN / 16;
constexpr int KPAD = BK + 2;    // row stride of a contraction-contiguous tile
constexpr int OPAD = 128 + 2;   // row stride of an outer-contiguous tile
constexpr int GROUP_M = 8;
constexpr int NUM_XCD = 8;

template <bool KC>
struct Tile {
    static constexpr int elems = KC ? 128 * KPAD : BK * OPAD;
};

// Global -> registers: 4 chunks of 2 doubles per thread.
// KC:  element (o, kk) of the tile is P[(o0 + o) * ld + k0 + kk]
// !KC: element (o, kk) of the tile is P[(k0 + kk) * ld + o0 + o]
// `fast` (uniform across the workgroup) says the whole 128 x 16 tile lies
// inside the operand and 16-byte loads are aligned: then the loads carry no
// per-element guard, so the compiler emits straight-line dwordx4 loads that
// stay in flight across the MFMAs of the current stage.  Edge tiles take the
// guarded path.
template <bool KC, bool FULL>
__device__ inline void load_tile(const double *__restrict__ P, int64_t ld, int o0, int k0,
                                 int oext, int kext, bool vec, double2 (&r)[4]) {
    const int tid = threadIdx.x;
    const bool fast = FULL || (vec && o0 + 128 <= oext && k0 + BK <= kext);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = tid + THREADS * i;
        int o, kk;
        if (KC) { o = c >> 3; kk = (c & 7) * 2; }
        else    { kk = c >> 6; o = (c & 63) * 2; }
        const int go = o0 + o, gk = k0 + kk;
        // the two elements of the chunk run along the contiguous index
        const int64_t base = KC ? (int64_t)go * ld + gk : (int64_t)gk * ld + go;
        if (fast) {
            r[i] = *reinterpret_cast<const double2 *>(P + base);
        } else {
            const bool in0 = go < oext && gk < kext;
            const bool in1 = KC ? (go < oext && gk + 1 < kext) : (gk < kext && go + 1 < oext);
            if (vec && in1) {
                r[i] = *reinterpret_cast<const double2 *>(P + base);
            } else {
                r[i].x = in0 ? P[base] : 0.0;
                r[i].y = in1 ? P[base + 1] : 0.0;
            }
        }
    }
}

template <bool KC>
__device__ inline void store_tile(double *__restrict__ L, const double2 (&r)[4]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = tid + THREADS * i;
        int off;
        if (KC) off = (c >> 3) * KPAD + (c & 7) * 2;
        else    off = (c >> 6) * OPAD + (c & 63) * 2;
        *reinterpret_cast<double2 *>(L + off) = r[i];
    }
}

// Fragments of k-step t of one stage: f[block] = the lane's element of
// MFMA block `block` (row or column wbase + 16*block + lane%16, k = 4j + t).
template <bool KC, int F>
__device__ inline void read_frags(const double *__restrict__ L, int wbase, int t, double (&f)[F]) {
    const int lane = threadIdx.x & 63;
    const int j = lane >> 4, l16 = lane & 15;
#pragma unroll
    for (int b = 0; b < F; ++b) {
        const int o = wbase + b * 16 + l16;
        f[b] = KC ? L[o * KPAD + 4 * j + t] : L[(4 * j + t) * OPAD + o];
    }
}

// ----- whole-tile path: no vector-ALU work in the main loop.  While the
// matrix cores are busy, VALU instructions of every wave on the SIMD get few
// issue slots, so the whole-tile loop keeps its address arithmetic scalar:
// each panel load is a uniform SGPR base (advanced by scalar arithmetic) plus
// the lane's fixed 32-bit byte offset, and the loop is unrolled over the two
// LDS buffers so every LDS access is a fixed register plus an immediate.

typedef __attribute__((address_space(1))) const char gchar;
typedef double d2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const d2v gd2v;

// A uniform global address computed on the vector ALU moved to scalar
// registers (kept in the global address space, so loads stay global loads).
__device__ __forceinline__ gchar *to_sgpr(const double *p) {
    const uint64_t u = (uint64_t)(uintptr_t)p;
    // the builtin returns int: widen through uint32_t (zero-extend)
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((unsigned)u);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (gchar *)(uintptr_t)(lo | (hi << 32));
}

// One operand's panel loads: stage kt's chunk i of this lane is at byte
// base + kt * step + i * istep + off.  Chunk i of a thread is chunk 0 moved
// by 32 tile rows (KC) or 4 k rows (!KC), a uniform stride, so one 32-bit
// lane offset serves all four.
struct Panel {
    gchar *base;
    int64_t step, istep;
    unsigned off;
};

template <bool KC>
__device__ __forceinline__ Panel make_panel(const double *P, int64_t ld, int o0) {
    Panel q;
    const unsigned tid = threadIdx.x;
    q.base = to_sgpr(KC ? P + (int64_t)o0 * ld : P + o0);
    q.step = KC ? (int64_t)BK * 8 : (int64_t)BK * ld * 8;
    q.istep = KC ? (int64_t)(THREADS / 8) * ld * 8 : (int64_t)(THREADS / 64) * ld * 8;
    // chunk 0: KC (o, kk) = (tid / 8, 2 (tid % 8)); !KC (kk, o) = (tid / 64, 2 (tid % 64))
    const unsigned ldu = (unsigned)ld;
    q.off = KC ? ((tid >> 3) * ldu + (tid & 7) * 2u) * 8u : ((tid >> 6) * ldu + (tid & 63) * 2u) * 8u;
    return q;
}

__device__ __forceinline__ void load_panel(const Panel &q, int kt, double2 (&r)[4]) {
    gchar *b = q.base + (int64_t)kt * q.step;
    // Redefine the offset here so its zero extension is not hoisted out of
    // the loop: the SGPR-base + 32-bit-offset load form needs to see it.
    unsigned off = q.off;
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // a native vector load (a HIP double2 copied from the global address
        // space would go through private memory)
        gchar *bi = b + i * q.istep;
        asm volatile("" : "+s"(bi));  // keep the chunk's base a scalar operand
        const d2v v = *reinterpret_cast<gd2v *>(bi + off);
        r[i].x = v.x;
        r[i].y = v.y;
    }
}

// One stage of the whole-tile loop reading LDS buffer CUR: loads of stage
// kt + 1 (the last stage reloads itself into the idle buffer), 3 k-steps of
// MFMAs, the loaded tiles stored to buffer CUR ^ 1, the last k-step, a
// barrier.
template <bool A_KC, bool B_KC, int CUR>
__device__ __forceinline__ void full_stage(int kt, int nk, const Panel &pa, const Panel &pb,
                                  double (*lds_a)[Tile<A_KC>::elems],
                                  double (*lds_b)[Tile<B_KC>::elems], int wm, int wn,
                                  d4 (&acc)[FM][FN]) {
    double2 ra[4], rb[4];
    const int knext = kt + 1 < nk ? kt + 1 : kt;
    load_panel(pa, knext, ra);
    load_panel(pb, knext, rb);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        // No wave reads buffer CUR ^ 1 during this stage (all passed the
        // previous barrier), so the loaded tiles go there before the last
        // k-step, whose MFMAs then cover the LDS writes.
        if (t == 3) {
            store_tile<A_KC>(lds_a[CUR ^ 1], ra);
            store_tile<B_KC>(lds_b[CUR ^ 1], rb);
            __builtin_amdgcn_sched_barrier(0);
        }
        double fa[FM], fb[FN];
        read_frags<A_KC, FM>(lds_a[CUR], wm * WM, t, fa);
        read_frags<B_KC, FN>(lds_b[CUR], wn * WN, t, fb);
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
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

// A_KC: op(A)'s contraction index is contiguous (trans_a == 0).
// B_KC: op(B)'s contraction index is contiguous (trans_b == 1).
// FULL: every tile is whole (edge tiles moved back inside the matrix, k a
// multiple of 16: the launcher adds a partial last stage separately) and
// both operands allow 16-byte loads; the loads then carry no guards, and the
// stores only skip the cells a moved tile shares with its neighbour.
template <bool A_KC, bool B_KC, bool FULL>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
gemm_f64_kernel(int m, int n, int k, const double *__restrict__ A, int64_t lda,
                const double *__restrict__ B, int64_t ldb, double *__restrict__ C, int64_t ldc,
                int vec_a, int vec_b, int accumulate, int kc = 0, int64_t cstride = 0) {
    __shared__ __attribute__((aligned(16))) double lds_a[2][Tile<A_KC>::elems];
    __shared__ __attribute__((aligned(16))) double lds_b[2][Tile<B_KC>::elems];

    // split contraction (kc > 0): workgroup row y of the grid multiplies the
    // chunk [y kc, (y + 1) kc) of k into its own partial product at C + y cstride
    if (kc > 0) {
        const int k0 = (int)blockIdx.y * kc;
        A += A_KC ? (int64_t)k0 : (int64_t)k0 * lda;
        B += B_KC ? (int64_t)k0 : (int64_t)k0 * ldb;
        C += (int64_t)blockIdx.y * cstride;
        k = min(kc, k - k0);
    }

    const int tiles_m = (m + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    // the cells this tile owns start at (rlo, clo); on the whole-tile path a
    // tile that would run past an edge is moved back to end at m (or n), so
    // it stays whole and in bounds, and stores only the cells it owns
    const int rlo = tm * BM, clo = tn * BN;
    const int m0 = FULL ? min(rlo, m - BM) : rlo, n0 = FULL ? min(clo, n - BN) : clo;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave & 1, wn = wave >> 1;

    d4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    const int nk = (k + BK - 1) / BK;
    if constexpr (FULL) {
        const Panel pa = make_panel<A_KC>(A, lda, m0);
        const Panel pb = make_panel<B_KC>(B, ldb, n0);
        {
            double2 ra[4], rb[4];
            load_panel(pa, 0, ra);
            load_panel(pb, 0, rb);
            store_tile<A_KC>(lds_a[0], ra);
            store_tile<B_KC>(lds_b[0], rb);
        }
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            full_stage<A_KC, B_KC, 0>(kt, nk, pa, pb, lds_a, lds_b, wm, wn, acc);
            if (kt + 1 < nk) full_stage<A_KC, B_KC, 1>(kt + 1, nk, pa, pb, lds_a, lds_b, wm, wn, acc);
        }
    } else {
    double2 ra[4], rb[4];
    load_tile<A_KC, FULL>(A, lda, m0, 0, m, k, vec_a, ra);
    load_tile<B_KC, FULL>(B, ldb, n0, 0, n, k, vec_b, rb);
    store_tile<A_KC>(lds_a[0], ra);
    store_tile<B_KC>(lds_b[0], rb);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        // The last stage reloads its own (in-bounds) tile and stores it to
        // the idle buffer, which no wave reads any more: loads and stores are
        // unconditional, so the compiler neither sinks the loads behind the
        // MFMAs nor keeps the staging registers in scratch.  The scheduling
        // barrier pins the loads ahead of the stage's MFMAs.
        const int knext = (more ? kt + 1 : kt) * BK;
        load_tile<A_KC, FULL>(A, lda, m0, knext, m, k, vec_a, ra);
        load_tile<B_KC, FULL>(B, ldb, n0, knext, n, k, vec_b, rb);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double fa[FM], fb[FN];
            read_frags<A_KC, FM>(lds_a[cur], wm * WM, t, fa);
            read_frags<B_KC, FN>(lds_b[cur], wn * WN, t, fb);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0,
                                                                     0);
        }
        store_tile<A_KC>(lds_a[cur ^ 1], ra);
        store_tile<B_KC>(lds_b[cur ^ 1], rb);
        __syncthreads();
    }
    }

    const int lane = threadIdx.x & 63;
    const int j = lane >> 4, l16 = lane & 15;
#pragma unroll
    for (int a = 0; a < FM; ++a) {
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int col = n0 + wn * WN + b * 16 + l16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + wm * WM + a * 16 + j + 4 * i;
                if (FULL ? (row >= rlo && col >= clo) : (row < m && col < n)) {
                    double *dst = C + (int64_t)row * ldc + col;
                    *dst = accumulate ? *dst + acc[a][b][i] : acc[a][b][i];
                }
            }
        }
    }
}

template <bool A_KC, bool B_KC>
hipError_t launch(int m, int n, int k, const double *A, int64_t lda, const double *B,
                  int64_t ldb, double *C, int64_t ldc, int accumulate, hipStream_t s) {
    const int tiles = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    const int vec_a = (lda % 2 == 0) && (((uintptr_t)A & 15) == 0);
    const int vec_b = (ldb % 2 == 0) && (((uintptr_t)B & 15) == 0);
    // the whole-tile path: 16-byte loads, at least one whole stage of k,
    // every lane's byte offset inside a stage's panel below 2^32, and m, n
    // at least one tile, so that edge tiles can be moved back to end at m
    // and n (a move along an operand's contiguous index must keep 16-byte
    // alignment: m, n even there)
    const int64_t span_a = (A_KC ? (int64_t)BM * lda : (int64_t)BK * lda) * 8;
    const int64_t span_b = (B_KC ? (int64_t)BN * ldb : (int64_t)BK * ldb) * 8;
    const bool full = vec_a && vec_b && m >= BM && n >= BN && k >= BK &&
                      (A_KC || m % 2 == 0) && (B_KC || n % 2 == 0) &&
                      span_a < ((int64_t)1 << 32) && span_b < ((int64_t)1 << 32);
    if (full) {
        // the whole 16-deep stages of k on the whole-tile path; a last
        // partial stage (k % 16 terms) is added to C by a guarded launch
        const int kf = k / BK * BK;
        {
            TraceScope ts(TCU_KERNEL_GEMM_F64, m, n, kf, 1, 2.0 * m * n * (double)kf, s);
            gemm_f64_kernel<A_KC, B_KC, true><<<tiles, THREADS, 0, s>>>(
                m, n, kf, A, lda, B, ldb, C, ldc, vec_a, vec_b, accumulate);
        }
        if (kf < k) {
            const double *At = A_KC ? A + kf : A + (int64_t)kf * lda;
            const double *Bt = B_KC ? B + kf : B + (int64_t)kf * ldb;
            TraceScope ts(TCU_KERNEL_GEMM_F64, m, n, k - kf, 1, 2.0 * m * n * (double)(k - kf), s);
            gemm_f64_kernel<A_KC, B_KC, false><<<tiles, THREADS, 0, s>>>(
                m, n, k - kf, At, lda, Bt, ldb, C, ldc, vec_a, vec_b, 1);
        }
    } else {
        TraceScope ts(TCU_KERNEL_GEMM_F64, m, n, k, 1, 2.0 * m * n * (double)k, s);
        gemm_f64_kernel<A_KC, B_KC, false><<<tiles, THREADS, 0, s>>>(m, n, k, A, lda, B, ldb, C,
                                                                     ldc, vec_a, vec_b, accumulate);
    }
    return hipGetLastError();
}

// The split contraction's partial products summed in chunk order:
// C[i, j] = sum_p part[p][i * n + j], the same order on every run.
__global__ void __launch_bounds__(THREADS)
sum_partials_kernel(int m, int n, int parts, const double *__restrict__ part,
                    double *__restrict__ C, int64_t ldc) {
    const int64_t i = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    const int64_t mn = (int64_t)m * n;
    if (i >= mn) return;
    double s = 0.0;
    for (int p = 0; p < parts; ++p) s += part[p * mn + i];
    C[(i / n) * ldc + i % n] = s;
}

// Chunks of the split contraction: enough workgroups for two rounds of the
// chip when the output alone has few tiles, each chunk at least 256 deep.
// 0: no split.
int split_parts(int m, int n, int k) {
    const int64_t tiles = (int64_t)((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    if (tiles >= 128 || k < 1024) return 0;
    int64_t parts = (512 + tiles - 1) / tiles;
    parts = std::min<int64_t>(parts, k / 256);
    return parts >= 2 ? (int)parts : 0;
}

int split_chunk(int k, int parts) { return ((k + parts - 1) / parts + BK - 1) / BK * BK; }

template <bool A_KC, bool B_KC>
hipError_t launch_split(int m, int n, int k, const double *A, int64_t lda, const double *B,
                        int64_t ldb, double *C, int64_t ldc, double *part, int parts,
                        hipStream_t s) {
    const int kc = split_chunk(k, parts);
    const int used = (k + kc - 1) / kc;  // chunks that hold part of k
    const int tiles = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    const int vec_a = (lda % 2 == 0) && (((uintptr_t)A & 15) == 0);
    const int vec_b = (ldb % 2 == 0) && (((uintptr_t)B & 15) == 0);
    {
        TraceScope ts(TCU_KERNEL_GEMM_F64, m, n, k, used, 2.0 * m * n * (double)k, s);
        gemm_f64_kernel<A_KC, B_KC, false><<<dim3(tiles, used), THREADS, 0, s>>>(
            m, n, k, A, lda, B, ldb, part, n, vec_a, vec_b, 0, kc, (int64_t)m * n);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t mn = (int64_t)m * n;
    sum_partials_kernel<<<(unsigned)((mn + THREADS - 1) / THREADS), THREADS, 0, s>>>(
        m, n, used, part, C, ldc);
    return hipGetLastError();
}

}  // namespace

size_t gemm_f64_split_bytes(int m, int n, int k) {
    const int parts = split_parts(m, n, k);
    return parts == 0 ? 0 : (size_t)parts * (size_t)m * (size_t)n * sizeof(double);
}

hipError_t launch_gemm_f64_split(int trans_a, int trans_b, int m, int n, int k, const double *A,
                                 int64_t lda, const double *B, int64_t ldb, double *C,
                                 int64_t ldc, double *part, hipStream_t s) {
    const int parts = split_parts(m, n, k);
    if (parts == 0 || part == nullptr)
        return launch_gemm_f64(trans_a, trans_b, m, n, k, A, lda, B, ldb, C, ldc, s);
    if (!trans_a && !trans_b)
        return launch_split<true, false>(m, n, k, A, lda, B, ldb, C, ldc, part, parts, s);
    if (!trans_a && trans_b)
        return launch_split<true, true>(m, n, k, A, lda, B, ldb, C, ldc, part, parts, s);
    if (trans_a && !trans_b)
        return launch_split<false, false>(m, n, k, A, lda, B, ldb, C, ldc, part, parts, s);
    return launch_split<false, true>(m, n, k, A, lda, B, ldb, C, ldc, part, parts, s);
}

int gemm_f64_row_cut(int m, int n) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 0;
    // two workgroups per CU: each is 4 waves, and the kernel runs 2 waves per SIMD
    const int64_t resident = 2 * (int64_t)cus;
    const int64_t rt = (m + BM - 1) / BM, ct = (n + BN - 1) / BN;
    auto rounds = [&](int64_t tiles) { return (tiles + resident - 1) / resident; };
    const int64_t whole = rounds(rt * ct);
    if (whole < 2) return 0;
    // the most even cut among those that add no round
    auto skew = [&](int64_t r) { return 2 * r > rt ? 2 * r - rt : rt - 2 * r; };
    int64_t best = 0;
    for (int64_t r = 1; r < rt; ++r) {
        if (rounds(r * ct) + rounds((rt - r) * ct) != whole) continue;
        if (best == 0 || skew(r) < skew(best)) best = r;
    }
    return (int)(best * BM);
}

hipError_t launch_gemm_f64(int trans_a, int trans_b, int m, int n, int k, const double *A,
                           int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                           hipStream_t s, int accumulate) {
    if (m == 0 || n == 0) return hipSuccess;
    if (!trans_a && !trans_b)
        return launch<true, false>(m, n, k, A, lda, B, ldb, C, ldc, accumulate, s);
    if (!trans_a && trans_b)
        return launch<true, true>(m, n, k, A, lda, B, ldb, C, ldc, accumulate, s);
    if (trans_a && !trans_b)
        return launch<false, false>(m, n, k, A, lda, B, ldb, C, ldc, accumulate, s);
    return launch<false, true>(m, n, k, A, lda, B, ldb, C, ldc, accumulate, s);
}

}  // namespace tcu
