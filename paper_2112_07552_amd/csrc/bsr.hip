// bsr.hip -- the join-aggregate on block-sparse encodings: the analogue of
// TCUDB's TCU-SpMM operator (Section 4.2.4, handling sparse matrices).
//
// When the key domain K is large and each group touches few keys (the
// microbenchmarks' many-distinct-values regime, Section 5.2), X (M x K) and
// Y (K x N) are almost all zeros and the dense product wastes its work on
// them.  Following the paper, both encodings are cut into 16 x 16 tiles, the
// tiles holding no record are never stored or multiplied, and the remaining
// tile pairs run on the matrix cores:
//
//   1. tile key per record: X: (g/16, k/16), Y: (h/16, k/16), packed as
//      outer << 32 | key tile;
//   2. the distinct tile keys, sorted, and each record's tile index (the
//      dictionary machinery of dict.hip: hash set, compaction, bitonic sort,
//      rank lookup; one host synchronisation to size the sort);
//   3. the first tile of every tile row of X and tile column of Y (binary
//      search over the sorted keys): tile lists sorted by key tile;
//   4. every record's value added into its tile (16 x 16 FP64, X tiles
//      [g%16][k%16], Y tiles [k%16][h%16]);
//   5. one wave per 16 x 16 tile of C: merge the key-tile lists of X's tile
//      row and Y's tile column and, for every common key tile, four
//      v_mfma_f64_16x16x4_f64 into the tile's accumulator; then store the
//      tile (zero where the lists do not meet).
// The result equals the dense operator's: the products skipped are products
// of all-zero tiles.  C is dense M x N FP64, as for tcu_join_agg_fwd.
#include "internal.h"

namespace tcu {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int TB = 16;                           // tile edge
constexpr long long kBadKey = 0x7fffffffffffffffll;  // record outside the shape

template <typename T>
__global__ void __launch_bounds__(kThreads)
tile_key_kernel(int64_t n, const int32_t *__restrict__ outer, const int32_t *__restrict__ key,
                int outer_ext, int key_ext, long long *__restrict__ keys, StatusBlock *st,
                int which) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const int o = outer[i], k = key[i];
        bad = (unsigned)o >= (unsigned)outer_ext || (unsigned)k >= (unsigned)key_ext;
        keys[i] = bad ? kBadKey : ((long long)(o / TB) << 32) | (long long)(k / TB);
    }
    const unsigned long long mask = __ballot(bad);
    if (mask != 0ull && (threadIdx.x & 63) == 0) {
        atomicOr(&st->flags, kFlagKeyRange);
        atomicAdd(which == 0 ? &st->skipped_a : &st->skipped_b,
                  (unsigned long long)__popcll(mask));
    }
}

// ptr[o] = index of the first sorted tile key whose outer tile is >= o.
__global__ void __launch_bounds__(kThreads)
tile_ptr_kernel(const long long *__restrict__ tkeys, int64_t ntiles, int outer_tiles,
                int *__restrict__ ptr) {
    const int o = blockIdx.x * kThreads + threadIdx.x;
    if (o > outer_tiles) return;
    const long long target = (long long)o << 32;
    int64_t lo = 0, hi = ntiles;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (tkeys[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    ptr[o] = (int)lo;
}

// tiles[code][r][c] (+)= v with (r, c) = (outer % 16, key % 16) for X, or
// (key % 16, outer % 16) for Y (key_rows).
template <typename T, bool UNIQUE>
__global__ void __launch_bounds__(kThreads)
tile_scatter_kernel(int64_t n, const int32_t *__restrict__ outer, const int32_t *__restrict__ key,
                    const T *__restrict__ val, const long long *__restrict__ keys,
                    const int *__restrict__ codes, int key_rows, double *__restrict__ tiles) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n || keys[i] == kBadKey) return;
    const int o = outer[i] % TB, k = key[i] % TB;
    const int cell = key_rows ? k * TB + o : o * TB + k;
    const double v = val ? (double)val[i] : 1.0;
    double *dst = tiles + (int64_t)codes[i] * (TB * TB) + cell;
    if (UNIQUE) *dst = v;
    else unsafeAtomicAdd(dst, v);
}

// One wave per output tile (gt, ht), tiles numbered row-major so that the
// waves of a workgroup store neighbouring 128-byte row segments of C.
__global__ void __launch_bounds__(kThreads)
bsr_product_kernel(int M, int N, int mt, int nt, const long long *__restrict__ xkeys,
                   const int *__restrict__ xptr, const double *__restrict__ xt,
                   const long long *__restrict__ ykeys, const int *__restrict__ yptr,
                   const double *__restrict__ yt, double *__restrict__ C, int64_t ldc) {
    const int64_t tile =
        (int64_t)blockIdx.x * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tile >= (int64_t)mt * nt) return;
    const int gt = (int)(tile / nt), ht = (int)(tile % nt);
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, q = lane >> 4;

    int xa = xptr[gt], xb = xptr[gt + 1];
    int ya = yptr[ht], yb = yptr[ht + 1];
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    while (xa < xb && ya < yb) {
        const int kx = (int)(xkeys[xa] & 0xffffffffll);
        const int ky = (int)(ykeys[ya] & 0xffffffffll);
        if (kx == ky) {
            const double *xp = xt + (int64_t)xa * (TB * TB);
            const double *yp = yt + (int64_t)ya * (TB * TB);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // A lane: X tile [r16][4t + q]; B lane: Y tile [4t + q][r16]
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xp[r16 * TB + 4 * t + q],
                                                           yp[(4 * t + q) * TB + r16], acc, 0, 0,
                                                           0);
            }
            ++xa;
            ++ya;
        } else if (kx < ky) {
            ++xa;
        } else {
            ++ya;
        }
    }
    // accumulator item i of lane l: row q + 4 i, column r16
    const int col = ht * TB + r16;
    if (col < N) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = gt * TB + q + 4 * i;
            if (row < M) C[(int64_t)row * ldc + col] = acc[i];
        }
    }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

struct Side {
    long long *keys;
    int *codes;
    long long *tkeys;
    int *ptr;
    double *tiles;
};

// distinct tile keys of n records: at most n, and at most every tile of the
// grid plus the one sentinel key of skipped records
inline int64_t max_tiles(int64_t n, int outer_ext, int key_ext) {
    const int64_t grid = (int64_t)((outer_ext + TB - 1) / TB) * ((key_ext + TB - 1) / TB) + 1;
    return n < grid ? n : grid;
}

struct Layout {
    size_t status, dict_ws, total;
    size_t keys[2], codes[2], tkeys[2], ptr[2], tiles[2];
};

Layout layout(int64_t na, int64_t nb, int M, int K, int N) {
    Layout L{};
    size_t off = sizeof(StatusBlock);
    L.status = 0;
    const int64_t n[2] = {na, nb};
    const int outer[2] = {M, N};
    for (int s = 0; s < 2; ++s) {
        L.keys[s] = off;
        off += align_up((size_t)n[s] * 8);
        L.codes[s] = off;
        off += align_up((size_t)n[s] * 4);
        L.tkeys[s] = off;
        off += align_up((size_t)(n[s] > 0 ? n[s] : 1) * 8);
        L.ptr[s] = off;
        off += align_up((size_t)((outer[s] + TB - 1) / TB + 1) * 4);
        L.tiles[s] = off;
        off += align_up((size_t)max_tiles(n[s], outer[s], K) * TB * TB * 8);
    }
    L.dict_ws = off;
    const int64_t nmax = na > nb ? na : nb;
    off += align_up(dict_workspace_bytes(nmax));
    L.total = off;
    return L;
}

template <typename T>
hipError_t scatter_t(const tcu_relation &R, const Side &sd, int key_rows, hipStream_t s) {
    const T *v = static_cast<const T *>(R.val);
    if (R.flags & TCU_REL_UNIQUE_CELLS)
        tile_scatter_kernel<T, true><<<grid_for(R.n), kThreads, 0, s>>>(
            R.n, R.group, R.key, v, sd.keys, sd.codes, key_rows, sd.tiles);
    else
        tile_scatter_kernel<T, false><<<grid_for(R.n), kThreads, 0, s>>>(
            R.n, R.group, R.key, v, sd.keys, sd.codes, key_rows, sd.tiles);
    return hipGetLastError();
}

// Steps 1-4 for one relation: outer = group column (g for A, h for B).
hipError_t build_side(const tcu_relation &R, int outer_ext, int K, int which, const Side &sd,
                      void *dict_ws, StatusBlock *st, hipStream_t s) {
    const int outer_tiles = (outer_ext + TB - 1) / TB;
    int64_t ntiles = 0;
    if (R.n > 0) {
        if (R.dtype == TCU_F32)
            tile_key_kernel<float><<<grid_for(R.n), kThreads, 0, s>>>(R.n, R.group, R.key,
                                                                      outer_ext, K, sd.keys, st,
                                                                      which);
        else
            tile_key_kernel<double><<<grid_for(R.n), kThreads, 0, s>>>(R.n, R.group, R.key,
                                                                       outer_ext, K, sd.keys, st,
                                                                       which);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = run_dict_encode(sd.keys, R.n, nullptr, 0, sd.codes, nullptr, sd.tkeys, &ntiles,
                            dict_ws, s);
        if (e != hipSuccess) return e;
        // the sentinel key of skipped records, if present, is the last tile
        // and lies beyond every tile row: the pointers exclude it
        e = launch_zero_f64(sd.tiles, (size_t)ntiles * TB * TB, s);
        if (e != hipSuccess) return e;
        e = R.dtype == TCU_F32 ? scatter_t<float>(R, sd, which, s)
                               : scatter_t<double>(R, sd, which, s);
        if (e != hipSuccess) return e;
    }
    tile_ptr_kernel<<<grid_for(outer_tiles + 1), kThreads, 0, s>>>(sd.tkeys, ntiles, outer_tiles,
                                                                   sd.ptr);
    return hipGetLastError();
}

}  // namespace

size_t bsr_workspace_bytes(int64_t na, int64_t nb, int M, int K, int N) {
    return layout(na, nb, M, K, N).total;
}

hipError_t run_join_agg_bsr(const tcu_relation &A, const tcu_relation &B, int M, int K, int N,
                            double *C, void *ws, hipStream_t s) {
    const Layout L = layout(A.n, B.n, M, K, N);
    char *base = static_cast<char *>(ws);
    StatusBlock *st = reinterpret_cast<StatusBlock *>(base);
    Side sd[2];
    for (int i = 0; i < 2; ++i) {
        sd[i].keys = reinterpret_cast<long long *>(base + L.keys[i]);
        sd[i].codes = reinterpret_cast<int *>(base + L.codes[i]);
        sd[i].tkeys = reinterpret_cast<long long *>(base + L.tkeys[i]);
        sd[i].ptr = reinterpret_cast<int *>(base + L.ptr[i]);
        sd[i].tiles = reinterpret_cast<double *>(base + L.tiles[i]);
    }
    hipError_t e = launch_clear_status(st, s);
    if (e != hipSuccess) return e;
    e = build_side(A, M, K, 0, sd[0], base + L.dict_ws, st, s);
    if (e != hipSuccess) return e;
    e = build_side(B, N, K, 1, sd[1], base + L.dict_ws, st, s);
    if (e != hipSuccess) return e;
    const int mt = (M + TB - 1) / TB, nt = (N + TB - 1) / TB;
    const int64_t waves = (int64_t)mt * nt;
    const int64_t blocks = (waves + 3) / 4;
    if (blocks > 0x7fffffffll) return hipErrorInvalidValue;
    bsr_product_kernel<<<(unsigned)blocks, kThreads, 0, s>>>(M, N, mt, nt, sd[0].tkeys,
                                                             sd[0].ptr, sd[0].tiles, sd[1].tkeys,
                                                             sd[1].ptr, sd[1].tiles, C, N);
    return hipGetLastError();
}

}  // namespace tcu
