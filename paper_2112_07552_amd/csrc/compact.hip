// compact.hip -- nonzero(): the matrix-to-table conversion between the
// joins of a multi-way join (TCUDB Section 3.2, query Q2).
//
// After the first join, the n x m result matrix is turned back into the
// list of its nonzero cells, (i, j) with M[i,j] != 0, in row-major order, so
// that the next join can re-encode the surviving tuple pairs.  This is an
// HBM-bound stream compaction over the whole matrix (8 bytes read per
// cell), done in three passes:
//   1. every workgroup counts the nonzeros of its chunk of 4096 cells;
//   2. one workgroup turns the chunk counts into exclusive offsets;
//   3. every workgroup re-reads its chunk and writes the (row, col) pairs of
//      its nonzeros at their offsets (wave ballots give the in-order rank of
//      each nonzero inside the chunk).
// Row-major order makes the output deterministic and identical to the
// order a sequential scan would give.  An optional column map replaces the
// column by map[col] in a third output (the key of the next join).
#include "internal.h"

namespace tcu {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr int kChunk = kThreads * kPerThread;  // cells per workgroup

// Row and column of flat cell index i, cols >= 1: the quotient from a
// multiply by the reciprocal, then corrected by one either way.  i < 2^43
// (the launch covers at most 2^31 chunks of 4096 cells), so i is exact in a
// double and the product is within 2^-8 of i / cols.
__device__ inline void row_col(int64_t i, int64_t cols, double inv_cols, int64_t &r, int64_t &c) {
    r = (int64_t)((double)i * inv_cols);
    c = i - r * cols;
    if (c < 0) { --r; c += cols; }
    if (c >= cols) { ++r; c -= cols; }
}

// The kPerThread cells of this thread, read before any is used: cell j is
// b * kChunk + j * kThreads + t.  Every lane loads (cell 0 stands in past the
// end, total > 0), so the loads are in flight together; contiguous matrices
// (ld == cols, a uniform branch) need no row/column split.
__device__ inline void load_cells(const double *__restrict__ M, int64_t total, int64_t cols,
                                  int64_t ld, double (&v)[kPerThread]) {
    const int64_t base = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    if (ld == cols) {
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const int64_t i = base + (int64_t)j * kThreads;
            const bool in = i < total;
            const double x = M[in ? i : 0];
            v[j] = in ? x : 0.0;
        }
    } else {
        const double inv = 1.0 / (double)cols;
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const int64_t i = base + (int64_t)j * kThreads;
            const bool in = i < total;
            int64_t r, c;
            row_col(in ? i : 0, cols, inv, r, c);
            const double x = M[r * ld + c];
            v[j] = in ? x : 0.0;
        }
    }
}

// Pass 1: nonzeros per chunk of kChunk cells (coalesced across the workgroup).
__global__ void __launch_bounds__(kThreads)
nz_count_kernel(const double *__restrict__ M, int64_t total, int64_t cols, int64_t ld,
                unsigned *__restrict__ counts) {
    __shared__ unsigned wave_sum[kThreads / 64];
    double v[kPerThread];
    load_cells(M, total, cols, ld, v);
    unsigned c = 0;
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) c += v[j] != 0.0;
    // wave reduction by lane shuffles
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) wave_sum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned s = 0;
        for (int w = 0; w < kThreads / 64; ++w) s += wave_sum[w];
        counts[blockIdx.x] = s;
    }
}

// Exclusive prefix sum of n counts into offsets (int64), total into
// offsets[n]; one workgroup, sequential over tiles of kThreads.
__global__ void __launch_bounds__(kThreads)
nz_scan_kernel(const unsigned *__restrict__ counts, int64_t n,
               unsigned long long *__restrict__ offsets) {
    __shared__ unsigned long long buf[kThreads];
    unsigned long long carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += kThreads) {
        const int64_t i = t0 + threadIdx.x;
        const unsigned long long v = i < n ? counts[i] : 0ull;
        buf[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan in LDS
        for (int off = 1; off < kThreads; off <<= 1) {
            const unsigned long long add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0ull;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) offsets[i] = carry + buf[threadIdx.x] - v;
        carry += buf[kThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[n] = carry;
}

// Pass 3: the position of a nonzero is its chunk's offset plus the number of
// nonzeros before it in the chunk (in row-major order, which is the order
// j-major, then thread id).
__global__ void __launch_bounds__(kThreads)
nz_write_kernel(const double *__restrict__ M, int64_t total, int64_t cols, int64_t ld,
                const unsigned long long *__restrict__ offsets, int64_t capacity,
                int32_t *__restrict__ out_row, int32_t *__restrict__ out_col,
                const int32_t *__restrict__ col_map, int32_t *__restrict__ out_key) {
    __shared__ unsigned wave_cnt[kThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned long long pos = offsets[blockIdx.x];
    const double inv_cols = 1.0 / (double)cols;
    double v[kPerThread];
    load_cells(M, total, cols, ld, v);
    for (int j = 0; j < kPerThread; ++j) {
        const int64_t i = base + (int64_t)j * kThreads + threadIdx.x;
        const bool nz = v[j] != 0.0;  // cells past the end read as 0
        const unsigned long long mask = __ballot(nz);
        if (lane == 0) wave_cnt[wave] = (unsigned)__popcll(mask);
        __syncthreads();
        unsigned before = 0;
        for (int w = 0; w < wave; ++w) before += wave_cnt[w];
        unsigned all = before;
        for (int w = wave; w < kThreads / 64; ++w) all += wave_cnt[w];
        if (nz) {
            const unsigned long long lower = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
            const unsigned long long p = pos + before + (unsigned)__popcll(lower);
            if ((int64_t)p < capacity) {
                int64_t r, c;
                row_col(i, cols, inv_cols, r, c);
                out_row[p] = (int32_t)r;
                out_col[p] = (int32_t)c;
                if (out_key != nullptr) out_key[p] = col_map[c];
            }
        }
        pos += all;
        __syncthreads();  // wave_cnt is rewritten by the next step
    }
}

inline size_t chunks_of(int64_t total) { return (size_t)((total + kChunk - 1) / kChunk); }

}  // namespace

size_t nonzero_workspace_bytes(int64_t rows, int64_t cols) {
    const size_t nb = chunks_of(rows * cols);
    return align_up(nb * 4) + align_up((nb + 1) * 8);
}

hipError_t run_nonzero(const double *M, int64_t rows, int64_t cols, int64_t ld, int32_t *out_row,
                       int32_t *out_col, const int32_t *col_map, int32_t *out_key,
                       int64_t capacity, int64_t *count, void *ws, hipStream_t s) {
    const int64_t total = rows * cols;
    const size_t nb = chunks_of(total);
    char *p = static_cast<char *>(ws);
    unsigned *counts = reinterpret_cast<unsigned *>(p);
    unsigned long long *offsets = reinterpret_cast<unsigned long long *>(p + align_up(nb * 4));
    if (nb > 0x7fffffffull) return hipErrorInvalidValue;
    if (nb > 0) {
        nz_count_kernel<<<(unsigned)nb, kThreads, 0, s>>>(M, total, cols, ld, counts);
        nz_scan_kernel<<<1, kThreads, 0, s>>>(counts, (int64_t)nb, offsets);
        nz_write_kernel<<<(unsigned)nb, kThreads, 0, s>>>(M, total, cols, ld, offsets, capacity,
                                                          out_row, out_col, col_map, out_key);
    } else {
        // no cells: offsets[0] = 0
        hipError_t e = launch_zero_f64(reinterpret_cast<double *>(offsets), 1, s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long host = 0;
    e = hipMemcpyAsync(&host, offsets + nb, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *count = (int64_t)host;
    return hipSuccess;
}

}  // namespace tcu
