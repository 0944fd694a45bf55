// encode.hip -- step a1 (encoding, Sections 3.1 and 3.3 of TCUDB) and the
// record gathers of the adjoint.
//
// The encoding places every record's value at its (group, key) cell of a
// dense row-major matrix; duplicate cells add up.  It is a scatter bound by
// random-access throughput: per record it reads 4 + 4 + sizeof(val) bytes
// and performs one 8-byte FP64 atomic add (no return) into the matrix,
// which the zero pass wrote beforehand, or one plain store when the caller
// declares the cells unique.  Unique coordinates (the measured workload)
// give the record values bit for bit, since 0 + v == v.
#include <algorithm>

#include "internal.h"

namespace tcu {
namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) zero_f64_kernel(double *__restrict__ p, size_t n,
                                                            int vec) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    const size_t t0 = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (vec) {
        // p is 16-byte aligned: 16-byte stores over the even prefix, then the odd tail
        const size_t n2 = n / 2;
        double2 *p2 = reinterpret_cast<double2 *>(p);
        for (size_t i = t0; i < n2; i += stride) p2[i] = make_double2(0.0, 0.0);
        if (t0 == 0 && (n & 1)) p[n - 1] = 0.0;
    } else {
        for (size_t i = t0; i < n; i += stride) p[i] = 0.0;
    }
}

__global__ void zero_status_kernel(StatusBlock *st, uint32_t slices) {
    uint32_t *w = reinterpret_cast<uint32_t *>(st);
    w[threadIdx.x] = threadIdx.x == 1 ? slices : 0u;  // 64 threads x 4 bytes; word 1 = slices
}

// The plan words of the status block before a mixed-form product's
// certificate: needs and normalised-sum maxima to zero.
__global__ void reset_plan_kernel(StatusBlock *st) {
    st->need_bits = 0;
    st->need_slices = 0;
    st->umax_a = 0;
    st->umax_b = 0;
    st->need_cert = 0;
    st->need_min = kNeedUncertified;
    for (int j = 0; j < kExcThresholds; ++j) st->exc_seg[j] = 0;
    st->exceptions = 0;
}

// The plan a mixed-form product ran with (slices = 0: FP64 fallback).
__global__ void set_plan_kernel(StatusBlock *st, uint32_t slices, uint32_t bits, uint32_t need,
                                int fallback, uint32_t exceptions) {
    st->slices = slices;
    st->bits = bits;
    st->need = need;
    st->exceptions = exceptions;
    if (fallback) st->flags |= kFlagFallback;
}

// Counts this wave's invalid records and adds them to the status block once
// (st == nullptr: a repeated pass whose skips were already counted).
__device__ inline void report_skips(bool bad, StatusBlock *st, int which) {
    const unsigned long long mask = __ballot(bad);
    if (st != nullptr && mask != 0ull && (threadIdx.x & 63) == 0) {
        atomicOr(&st->flags, kFlagKeyRange);
        atomicAdd(which == 0 ? &st->skipped_a : &st->skipped_b,
                  (unsigned long long)__popcll(mask));
    }
}

// UNIQUE: the caller promised unique (group, key) cells, so a plain store
// replaces the atomic add (random 8-byte stores run about 3x faster than
// device-scope FP64 atomics, which fetch the whole line first).
template <typename T, bool UNIQUE>
__global__ void __launch_bounds__(kThreads)
encode_kernel(int64_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ key,
              const T *__restrict__ val, int transpose, int rows, int cols,
              double *__restrict__ out, StatusBlock *st, int which) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const int g = grp[i], k = key[i];
        const int r = transpose ? k : g;
        const int c = transpose ? g : k;
        if ((unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols) {
            const double v = val ? (double)val[i] : 1.0;
            double *dst = out + (size_t)r * (size_t)cols + c;
            if (UNIQUE) *dst = v;
            else unsafeAtomicAdd(dst, v);
        } else {
            bad = true;
        }
    }
    report_skips(bad, st, which);
}

__global__ void __launch_bounds__(kThreads)
gather_kernel(int64_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ key,
              int transpose, int rows, int cols, int r0, int r1, const double *__restrict__ src,
              double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int g = grp[i], k = key[i];
    const int r = transpose ? k : g;
    const int c = transpose ? g : k;
    const bool valid = (unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols;
    // a launch covers the records whose row lies in [r0, r1); the one that
    // starts at row 0 also writes the zeros of records outside the matrix
    if (valid ? (r < r0 || r >= r1) : r0 != 0) return;
    dst[i] = valid ? src[(size_t)r * (size_t)cols + c] : 0.0;
}

// ------------------------------------------------------- windowed scatter
// Random 8-byte stores into a matrix far larger than the last-level cache run
// at about a third of the rate they reach when the matrix stays cached (2^30
// records into an 8 GiB matrix: 50.8 ms; the same records one 128 MiB window
// of rows at a time, each window zeroed right before its records land: 16.5
// ms).  Large encodings therefore partition the records by row window first:
//   1. each workgroup counts its 8192 records per window (LDS histogram) into
//      a table, each count rounded up to a whole number of 32-slot runs;
//   2. per window, an exclusive scan of the table over the workgroups, then
//      one over the windows' totals: every (window, workgroup) run gets its
//      place, with no global atomics;
//   3. each workgroup writes its records' cell offsets inside their windows
//      (and values) into its runs, the unused slots of a run marked empty, so
//      that every 128-byte line of the scratch is written whole by one
//      workgroup;
//   4. each window is zeroed, then filled from its slots.
constexpr size_t kWindowBytes = (size_t)128 << 20;
constexpr size_t kWindowMinMatrix = (size_t)1 << 30;
constexpr int kMaxWindows = 1024;
constexpr int kPartThreads = 1024;
constexpr int kPartPer = 8;
constexpr int kPartChunk = kPartThreads * kPartPer;  // records per workgroup
static_assert(kPartThreads == kMaxWindows, "the partition pass scans its window counts in LDS");
constexpr unsigned kRun = 32;                         // slots per line of cell offsets
constexpr uint32_t kNoCell = 0xffffffffu;

__device__ inline bool record_cell(const int32_t *__restrict__ grp,
                                   const int32_t *__restrict__ key, int64_t i, int transpose,
                                   int rows, int cols, int &r, int &c) {
    const int g = grp[i], k = key[i];
    r = transpose ? k : g;
    c = transpose ? g : k;
    return (unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols;
}

__device__ inline unsigned round_run(unsigned x) { return (x + kRun - 1) / kRun * kRun; }

// Step 1: slots[b * nwg + wg] = the workgroup's records in window b, rounded
// up to whole runs; invalid records are counted as skips here, once.
__global__ void __launch_bounds__(kPartThreads)
window_count_kernel(int64_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ key,
                    int transpose, int rows, int cols, int wrows, int nw, int nwg,
                    uint32_t *__restrict__ slots, StatusBlock *st, int which) {
    __shared__ unsigned int hist[kMaxWindows];
    for (int b = threadIdx.x; b < nw; b += kPartThreads) hist[b] = 0u;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kPartChunk + threadIdx.x;
    unsigned bad = 0;
#pragma unroll
    for (int j = 0; j < kPartPer; ++j) {
        const int64_t i = i0 + (int64_t)j * kPartThreads;
        if (i < n) {
            int r, c;
            if (record_cell(grp, key, i, transpose, rows, cols, r, c))
                atomicAdd(&hist[r / wrows], 1u);
            else
                ++bad;
        }
    }
    if (bad != 0u && st != nullptr) {
        atomicOr(&st->flags, kFlagKeyRange);
        atomicAdd(which == 0 ? &st->skipped_a : &st->skipped_b, (unsigned long long)bad);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nw; b += kPartThreads)
        slots[(size_t)b * nwg + blockIdx.x] = round_run(hist[b]);
}

// Inclusive Hillis-Steele scan of v[0 .. kMaxWindows) in LDS (all threads of
// a kMaxWindows-thread workgroup take part).
__device__ inline void lds_scan(unsigned long long *v) {
    const int t = threadIdx.x;
    for (int d = 1; d < kMaxWindows; d <<= 1) {
        const unsigned long long add = t >= d ? v[t - d] : 0ull;
        __syncthreads();
        v[t] += add;
        __syncthreads();
    }
}

// Step 2a, one workgroup per window b: slots[b * nwg + w] becomes the
// exclusive prefix over w (each thread scans a contiguous segment), and
// totals[b] the window's slot count.
__global__ void __launch_bounds__(kMaxWindows)
window_runs_scan_kernel(uint32_t *__restrict__ slots, int nwg,
                        unsigned long long *__restrict__ totals) {
    __shared__ unsigned long long v[kMaxWindows];
    uint32_t *row = slots + (size_t)blockIdx.x * nwg;
    const int t = threadIdx.x;
    const int seg = (nwg + kMaxWindows - 1) / kMaxWindows;
    const int lo = t * seg, hi = min(nwg, lo + seg);
    unsigned long long sum = 0;
    for (int w = lo; w < hi; ++w) sum += row[w];
    v[t] = sum;
    __syncthreads();
    lds_scan(v);
    unsigned long long acc = v[t] - sum;  // exclusive prefix of this segment
    for (int w = lo; w < hi; ++w) {
        const uint32_t c = row[w];
        row[w] = (uint32_t)acc;  // a window's slots of one call stay below 2^32
        acc += c;
    }
    if (t == kMaxWindows - 1) totals[blockIdx.x] = v[t];
}

// Step 2b: offsets[b] = slots of the windows before b, b = 0..nw.
__global__ void __launch_bounds__(kMaxWindows)
window_scan_kernel(const unsigned long long *__restrict__ totals,
                   unsigned long long *__restrict__ offsets, int nw) {
    __shared__ unsigned long long v[kMaxWindows];
    const int t = threadIdx.x;
    v[t] = t < nw ? totals[t] : 0ull;
    __syncthreads();
    lds_scan(v);
    if (t < nw) offsets[t] = t == 0 ? 0ull : v[t - 1];
    if (t == nw - 1) offsets[nw] = v[t];
}

// Step 3: the same 8192 records per workgroup as step 1, ranked within their
// windows (LDS atomics), staged in LDS in window order, then written out so
// that consecutive threads fill consecutive slots of a run.
template <typename T>
__global__ void __launch_bounds__(kPartThreads)
window_partition_kernel(int64_t n, const int32_t *__restrict__ grp,
                        const int32_t *__restrict__ key, const T *__restrict__ val, int transpose,
                        int rows, int cols, int wrows, int nw, int nwg,
                        const uint32_t *__restrict__ runs,
                        const unsigned long long *__restrict__ offsets,
                        uint32_t *__restrict__ out_cell, T *__restrict__ out_val) {
    __shared__ unsigned int cnt[kMaxWindows];
    __shared__ unsigned long long base[kMaxWindows];
    __shared__ unsigned long long first[kMaxWindows];  // inclusive scan of cnt
    __shared__ uint32_t s_cell[kPartChunk];
    __shared__ T s_val[kPartChunk];
    __shared__ uint16_t s_bin[kPartChunk];
    const int t = threadIdx.x;
    for (int b = t; b < nw; b += kPartThreads) {
        cnt[b] = 0u;
        base[b] = offsets[b] + runs[(size_t)b * nwg + blockIdx.x];
    }
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kPartChunk + t;
    int bin[kPartPer];
    unsigned rank[kPartPer], cell[kPartPer];
    T v[kPartPer];
#pragma unroll
    for (int j = 0; j < kPartPer; ++j) {
        const int64_t i = i0 + (int64_t)j * kPartThreads;
        bin[j] = -1;
        rank[j] = 0u;
        cell[j] = 0u;
        v[j] = T(1);
        int r, c;
        if (i < n && record_cell(grp, key, i, transpose, rows, cols, r, c)) {
            const int b = r / wrows;
            bin[j] = b;
            // wrows * cols cells per window fit 32 bits (checked on the host)
            cell[j] = (unsigned)((size_t)(r - b * wrows) * (size_t)cols + (size_t)c);
            if (val != nullptr) v[j] = val[i];
            rank[j] = atomicAdd(&cnt[b], 1u);
        }
    }
    __syncthreads();
    // window b's records occupy staged positions [first[b] - cnt[b], first[b])
    first[t] = t < nw ? cnt[t] : 0u;  // kPartThreads == kMaxWindows
    __syncthreads();
    lds_scan(first);
#pragma unroll
    for (int j = 0; j < kPartPer; ++j) {
        if (bin[j] < 0) continue;
        const unsigned p = (unsigned)(first[bin[j]] - cnt[bin[j]]) + rank[j];
        s_cell[p] = cell[j];
        s_val[p] = v[j];
        s_bin[p] = (uint16_t)bin[j];
    }
    __syncthreads();
    const unsigned total = (unsigned)first[kMaxWindows - 1];
    for (unsigned p = t; p < total; p += kPartThreads) {
        const int b = s_bin[p];
        const unsigned long long q = base[b] + (p - (unsigned)(first[b] - cnt[b]));
        out_cell[q] = s_cell[p];
        if (out_val != nullptr) out_val[q] = s_val[p];
    }
    // the unused tail of each run: marked empty
    for (int x = t; x < nw * (int)kRun; x += kPartThreads) {
        const int b = x / (int)kRun;
        const unsigned s = cnt[b] + (unsigned)(x % (int)kRun);
        if (s < round_run(cnt[b])) out_cell[base[b] + s] = kNoCell;
    }
}

// Step 4: the slots of window w into its rows (out points at the window's
// first row, zeroed just before).
template <typename T, bool UNIQUE>
__global__ void __launch_bounds__(kThreads)
window_scatter_kernel(const unsigned long long *__restrict__ offsets, int w,
                      const uint32_t *__restrict__ cell, const T *__restrict__ val,
                      double *__restrict__ out) {
    const unsigned long long lo = offsets[w], hi = offsets[w + 1];
    const unsigned long long stride = (unsigned long long)gridDim.x * kThreads;
    for (unsigned long long i = lo + (unsigned long long)blockIdx.x * kThreads + threadIdx.x;
         i < hi; i += stride) {
        const uint32_t c = cell[i];
        if (c == kNoCell) continue;
        const double v = val != nullptr ? (double)val[i] : 1.0;
        if (UNIQUE) out[c] = v;
        else unsafeAtomicAdd(out + c, v);
    }
}

__global__ void __launch_bounds__(kThreads)
f64_to_i32_kernel(const double *__restrict__ src, int32_t *__restrict__ dst, size_t n,
                  StatusBlock *st) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    bool over = false;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const double v = src[i];
        const bool big = !(v <= 2147483647.0);
        over |= big;
        dst[i] = big ? 2147483647 : (int32_t)v;
    }
    if (__ballot(over) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&st->flags, kFlagCountRange);
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

inline unsigned capped_grid(size_t n) {
    size_t g = (n + kThreads - 1) / kThreads;
    const size_t cap = 256 * 64;  // 64 blocks per CU is plenty for a stream
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_zero_f64(double *p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int vec = ((uintptr_t)p & 15) == 0;
    zero_f64_kernel<<<capped_grid(vec ? n / 2 + 1 : n), kThreads, 0, s>>>(p, n, vec);
    return hipGetLastError();
}

hipError_t launch_clear_status(StatusBlock *st, hipStream_t s, uint32_t slices) {
    zero_status_kernel<<<1, 64, 0, s>>>(st, slices);
    return hipGetLastError();
}

hipError_t launch_reset_plan(StatusBlock *st, hipStream_t s) {
    reset_plan_kernel<<<1, 1, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_set_plan(StatusBlock *st, uint32_t slices, uint32_t bits, uint32_t need,
                           bool fallback, hipStream_t s, uint32_t exceptions) {
    set_plan_kernel<<<1, 1, 0, s>>>(st, slices, bits, need, fallback ? 1 : 0, exceptions);
    return hipGetLastError();
}

hipError_t launch_encode(const tcu_relation &R, int transpose, int rows, int cols, double *out,
                         StatusBlock *st, int which, hipStream_t s) {
    if (R.n == 0) return hipSuccess;
    const unsigned grid = grid_for(R.n);
    // algorithmic bytes: the record (group, key, value) in, one 8-byte cell out
    const double vbytes = R.val == nullptr ? 0.0 : (R.dtype == TCU_F32 ? 4.0 : 8.0);
    TraceScope ts(TCU_KERNEL_ENCODE, rows, cols, 0, 1, (double)R.n * (16.0 + vbytes), s);
    const bool unique = (R.flags & TCU_REL_UNIQUE_CELLS) != 0;
    const float *vf = static_cast<const float *>(R.val);
    const double *vd = static_cast<const double *>(R.val);
    if (R.dtype == TCU_F32) {
        if (unique)
            encode_kernel<float, true><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vf,
                                                                 transpose, rows, cols, out, st,
                                                                 which);
        else
            encode_kernel<float, false><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vf,
                                                                  transpose, rows, cols, out, st,
                                                                  which);
    } else {
        if (unique)
            encode_kernel<double, true><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vd,
                                                                  transpose, rows, cols, out, st,
                                                                  which);
        else
            encode_kernel<double, false><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vd,
                                                                   transpose, rows, cols, out,
                                                                   st, which);
    }
    return hipGetLastError();
}

namespace {

struct WindowPlan {
    int wrows = 0, nw = 0;
};

WindowPlan window_plan(int rows, int cols) {
    WindowPlan w;
    const size_t row_bytes = (size_t)cols * sizeof(double);
    int64_t wr = (int64_t)std::max<size_t>(1, kWindowBytes / row_bytes);
    wr = std::min<int64_t>(wr, rows);
    // at most kMaxWindows windows: wider ones for taller matrices
    wr = std::max<int64_t>(wr, ((int64_t)rows + kMaxWindows - 1) / kMaxWindows);
    w.wrows = (int)wr;
    w.nw = (int)(((int64_t)rows + wr - 1) / wr);
    return w;
}

size_t value_bytes(const tcu_relation &R) {
    return R.val == nullptr ? 0 : (R.dtype == TCU_F32 ? 4 : 8);
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Scratch: window totals and offsets (u64), the run table (u32, windows x
// workgroups), then per slot a cell offset (u32) and a value (the relation's
// value type).  Slots: the records plus at most kRun - 1 per run.
constexpr size_t kWindowHeader = (2 * (size_t)kMaxWindows + 1) * sizeof(unsigned long long);

struct WindowScratch {
    size_t table = 0, slots = 0, bytes = 0;
};

WindowScratch window_scratch(int64_t n, int nw, size_t vbytes) {
    WindowScratch w;
    const size_t nwg = (size_t)((n + kPartChunk - 1) / kPartChunk);
    w.table = (size_t)nw * nwg;
    w.slots = (size_t)n + w.table * (kRun - 1);
    w.bytes = align256(kWindowHeader) + align256(w.table * 4) + align256(w.slots * 4) +
              align256(w.slots * vbytes);
    return w;
}

template <typename T>
hipError_t encode_windowed(const tcu_relation &R, const T *val, int transpose, int rows, int cols,
                           double *out, StatusBlock *st, int which, void *scratch,
                           hipStream_t s) {
    const WindowPlan w = window_plan(rows, cols);
    const WindowScratch ws = window_scratch(R.n, w.nw, value_bytes(R));
    const int nwg = (int)((R.n + kPartChunk - 1) / kPartChunk);
    auto *totals = static_cast<unsigned long long *>(scratch);
    unsigned long long *offsets = totals + kMaxWindows;
    char *p = static_cast<char *>(scratch) + align256(kWindowHeader);
    auto *runs = reinterpret_cast<uint32_t *>(p);
    p += align256(ws.table * 4);
    auto *cell = reinterpret_cast<uint32_t *>(p);
    p += align256(ws.slots * 4);
    T *vals = val == nullptr ? nullptr : reinterpret_cast<T *>(p);
    window_count_kernel<<<(unsigned)nwg, kPartThreads, 0, s>>>(
        R.n, R.group, R.key, transpose, rows, cols, w.wrows, w.nw, nwg, runs, st, which);
    window_runs_scan_kernel<<<(unsigned)w.nw, kMaxWindows, 0, s>>>(runs, nwg, totals);
    window_scan_kernel<<<1, kMaxWindows, 0, s>>>(totals, offsets, w.nw);
    window_partition_kernel<T><<<(unsigned)nwg, kPartThreads, 0, s>>>(
        R.n, R.group, R.key, val, transpose, rows, cols, w.wrows, w.nw, nwg, runs, offsets, cell,
        vals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // each window's grid covers about twice its share of the slots; the
    // kernel loops over whatever its window holds
    const int64_t per = (int64_t)(ws.slots / (size_t)w.nw) + 1;
    const unsigned wgrid = (unsigned)std::min<int64_t>(
        65536, std::max<int64_t>(64, (2 * per + kThreads - 1) / kThreads));
    const bool unique = (R.flags & TCU_REL_UNIQUE_CELLS) != 0;
    for (int b = 0; b < w.nw; ++b) {
        const int r0 = b * w.wrows, nr = std::min(w.wrows, rows - r0);
        double *o = out + (size_t)r0 * (size_t)cols;
        if ((e = launch_zero_f64(o, (size_t)nr * (size_t)cols, s)) != hipSuccess) return e;
        if (unique)
            window_scatter_kernel<T, true><<<wgrid, kThreads, 0, s>>>(offsets, b, cell, vals, o);
        else
            window_scatter_kernel<T, false><<<wgrid, kThreads, 0, s>>>(offsets, b, cell, vals, o);
    }
    return hipGetLastError();
}

}  // namespace

size_t encode_scratch_bytes(const tcu_relation &R, int rows, int cols) {
    if (rows < 1 || cols < 1 || R.n < 1) return 0;
    if ((size_t)rows * (size_t)cols * sizeof(double) < kWindowMinMatrix) return 0;
    const WindowPlan w = window_plan(rows, cols);
    // cell offsets inside a window are 32-bit, and so are the run offsets
    // inside one window
    if (w.nw < 2 || (size_t)w.wrows * (size_t)cols > 0xfffffffeull) return 0;
    const WindowScratch ws = window_scratch(R.n, w.nw, value_bytes(R));
    if (ws.slots > 0xffffffffull) return 0;
    return ws.bytes;
}

hipError_t launch_encode_zeroed(const tcu_relation &R, int transpose, int rows, int cols,
                                double *out, StatusBlock *st, int which, void *scratch,
                                size_t scratch_bytes, hipStream_t s) {
    const size_t need = encode_scratch_bytes(R, rows, cols);
    if (need == 0 || scratch == nullptr || scratch_bytes < need ||
        ((uintptr_t)scratch & 255) != 0) {
        hipError_t e = launch_zero_f64(out, (size_t)rows * (size_t)cols, s);
        if (e == hipSuccess) e = launch_encode(R, transpose, rows, cols, out, st, which, s);
        return e;
    }
    const double vbytes = (double)value_bytes(R);
    // the launch record's plane count is the number of row windows
    TraceScope ts(TCU_KERNEL_ENCODE, rows, cols, 0, window_plan(rows, cols).nw,
                  (double)R.n * (16.0 + vbytes), s);
    if (R.val == nullptr)
        return encode_windowed<double>(R, nullptr, transpose, rows, cols, out, st, which,
                                       scratch, s);
    if (R.dtype == TCU_F32)
        return encode_windowed<float>(R, static_cast<const float *>(R.val), transpose, rows,
                                      cols, out, st, which, scratch, s);
    return encode_windowed<double>(R, static_cast<const double *>(R.val), transpose, rows, cols,
                                   out, st, which, scratch, s);
}

hipError_t launch_gather(const tcu_relation &R, int transpose, int rows, int cols,
                         const double *src, double *dst, hipStream_t s, int r0, int r1) {
    if (R.n == 0) return hipSuccess;
    if (r1 < 0) r1 = rows;
    // algorithmic bytes: group and key in, one 8-byte cell in, 8 bytes out
    TraceScope ts(TCU_KERNEL_GATHER, rows, cols, 0, 1, (double)R.n * 24.0, s);
    gather_kernel<<<grid_for(R.n), kThreads, 0, s>>>(R.n, R.group, R.key, transpose, rows, cols,
                                                     r0, r1, src, dst);
    return hipGetLastError();
}

hipError_t launch_f64_to_i32(const double *src, int32_t *dst, size_t n, StatusBlock *st,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    f64_to_i32_kernel<<<capped_grid(n), kThreads, 0, s>>>(src, dst, n, st);
    return hipGetLastError();
}

}  // namespace tcu
