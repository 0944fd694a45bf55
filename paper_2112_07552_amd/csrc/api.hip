// api.hip -- the C ABI of libtcudb.so (declared in include/tcudb.h).
//
// Host code only: argument checks, workspace layout, and the order of the
// kernel launches that make up the operator of TCUDB Section 3.3:
//   encode A -> X, encode B -> Y (Sections 3.1/3.3), C = X * Y (Lemma Q3),
// and its adjoint.  Every launch goes to the caller's stream.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

using namespace tcu;

namespace {

tcu_status hip_status(hipError_t e) { return e == hipSuccess ? TCU_OK : TCU_ERR_HIP; }

#define TCU_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_status(e_);    \
    } while (0)

bool relation_ok(const tcu_relation *R) {
    if (R == nullptr || R->n < 0) return false;
    if (R->n > 0 && (R->group == nullptr || R->key == nullptr)) return false;
    if ((R->flags & ~TCU_REL_UNIQUE_CELLS) != 0) return false;
    return R->dtype == TCU_F64 || R->dtype == TCU_F32;
}

bool shapes_ok(int32_t M, int32_t K, int32_t N) { return M >= 1 && K >= 1 && N >= 1; }

bool is_split(tcu_precision p) {
    return p == TCU_PREC_SPLIT_BF16 || p == TCU_PREC_SPLIT_I8 || p == TCU_PREC_CRT_I8;
}
bool is_crt(tcu_precision p) { return p == TCU_PREC_CRT_I8; }

bool precision_ok(tcu_precision p) { return p == TCU_PREC_FP64 || is_split(p); }

size_t pad128(int64_t x) { return (size_t)((x + 127) / 128 * 128); }
size_t pad64(int64_t x) { return (size_t)((x + 63) / 64 * 64); }
size_t pad256(int64_t x) { return (size_t)((x + 255) / 256 * 256); }
// Line padding of the int8 planes of the residue form and the certificate:
// the left operand's lines to the tile's 256 rows, the right operand's to the
// columns of the tile its product uses (its lines are the product's columns).
size_t padB(int64_t x) {
    const int64_t a = crt_tile_cols(x);
    return (size_t)((x + a - 1) / a * a);
}
size_t maxz(size_t a, size_t b) { return a > b ? a : b; }

// Mixed forms: tolerances below 2^-50 are refused (the encodings carry 53
// bits), and the residue form's int32 sums stay exact for k < 2^17.
constexpr double kMinTol = 0x1p-50;
constexpr int32_t kCrtMaxK = 131071;

double tol_or_default(double tol) { return tol > 0.0 ? tol : 1e-12; }

// Whether a mixed-form product of contraction length k can meet tol for
// some data (the shape-only part of the plan).
bool mixed_shape_ok(tcu_precision p, int32_t k, double tol) {
    return tol_or_default(tol) >= kMinTol && !(is_crt(p) && k > kCrtMaxK);
}

// FP64 additions in the digit forms' combination of one output: S
// diagonals per exact chunk of the contraction.
int64_t digit_adds(int S, bool bf16, int64_t k) {
    const int kstep = bf16 ? 16 : 32;
    const int64_t nblk = (int64_t)pad64(k) / kstep;
    const int64_t chunk = split_chunk_steps(S, bf16);
    return (int64_t)S * ((nblk + chunk - 1) / chunk);
}

// Step a0 host part: the plan of one product from its certificate (see
// tcudb.h, tcu_mixed_plan).
int mixed_plan(tcu_precision p, int32_t k, double tol, uint32_t need, double u,
               int32_t *bits_out) {
    if (!is_split(p) || k < 1) return TCU_ERR_ARG;
    tol = tol_or_default(tol);
    if (!mixed_shape_ok(p, k, tol) || need >= kNeedUncertified) return TCU_ERR_INFEASIBLE;
    if (!is_crt(p)) {
        const int S = need < 1 ? 1 : (int)need;
        return S <= TCU_MAX_SLICES ? S : TCU_ERR_INFEASIBLE;
    }
    const int b = need < 1 ? 1 : (int)need;
    if (b > 53) return TCU_ERR_INFEASIBLE;
    // |P| < 2^(2b) min(u, k); the reconstruction finds q = round(S / M) to
    // within 2^-40, so it needs M > 2 |P| (1 + 2^-38); 1e-6 bits is a factor
    // 1 + 6.9e-7, which also covers the roundings of the logarithms
    const double U = std::min(std::max(u, 1.0), (double)k);
    const double need_bits = 2.0 * b + log2(U) + 1.0 + 1e-6;
    for (int L = 1; L <= crt_max_moduli(); ++L)
        if (crt_modulus_bits(L) > need_bits) {
            if (bits_out != nullptr) *bits_out = b;
            return L;
        }
    return TCU_ERR_INFEASIBLE;
}

// Workspace layout:
//   [status block][X: M*K f64][Y: K*N f64]
//   [G: M*K f64][G2: K*N f64]                           (backward: dX, dY)
//   mixed forms, per operand A and B of a product:
//   [line maxima][exponents][normalised sums of |z|][partial column sums]
//   [magnitude plane][digit slices or residues, TCU_MAX_SLICES or
//    TCU_MAX_MODULI planes]  and, for the residue form, the product's residues
// In the mixed forms "A" is the left operand of a product (X forward, W
// for dX, X^T for dY) and "B" the right one (Y, Y^T, W).
struct Layout {
    size_t x = 0, y = 0, g = 0, g2 = 0, mba = 0, mbb = 0, ea = 0, eb = 0, sa = 0, sb = 0, res = 0;
    size_t sxa = 0, sxb = 0, psa = 0, psb = 0, qa = 0, qb = 0;
    size_t gsplit = 0, gsplit_bytes = 0;  // FP64 form: partial products of a split contraction
    size_t need = 0, exc = 0;  // residue form: per-cell needs, exception list
    size_t total = 0;
};

// Cells per segment of a residue-form product's exception list.
constexpr uint32_t kExcCap = 4096;

// Padding of the magnitude planes (the int8 GEMM's operand layout).
size_t qlen(int64_t x) { return (size_t)((x + crt_len_align() - 1) / crt_len_align() * crt_len_align()); }

// Whether a forward with a count output takes the int8 path (both relations
// with unique cells: multiplicities 0 or 1), which needs 0/1 planes.
bool count_planes(const tcu_relation *A, const tcu_relation *B, int flags) {
    if ((flags & TCU_WS_COUNT) == 0) return false;
    if (A == nullptr || B == nullptr) return true;
    return (A->flags & TCU_REL_UNIQUE_CELLS) && (B->flags & TCU_REL_UNIQUE_CELLS);
}

Layout plan_layout(int32_t M, int32_t K, int32_t N, tcu_precision p, int flags,
                   bool with_count_planes = false) {
    Layout L;
    const bool bwd = (flags & TCU_WS_BACKWARD) != 0;
    size_t off = sizeof(StatusBlock);
    L.x = off;
    off += align_up((size_t)M * (size_t)K * sizeof(double));
    L.y = off;
    off += align_up((size_t)K * (size_t)N * sizeof(double));
    if (bwd) {
        L.g = off;
        off += align_up((size_t)M * (size_t)K * sizeof(double));
        L.g2 = off;
        off += align_up((size_t)K * (size_t)N * sizeof(double));
    }
    if (is_split(p)) {
        const size_t digit = p == TCU_PREC_SPLIT_BF16 ? 2 : 1;
        const size_t planes = is_crt(p) ? TCU_MAX_MODULI : TCU_MAX_SLICES;
        auto padlA = [&](int64_t x) { return is_crt(p) ? pad256(x) : pad128(x); };
        auto padlB = [&](int64_t x) { return is_crt(p) ? padB(x) : pad128(x); };
        auto padk = [&](int64_t x) {
            const int64_t a = is_crt(p) ? crt_len_align() : 64;
            return (size_t)((x + a - 1) / a * a);
        };
        // (lines, length) of each operand: forward X (M, K) and Y (N, K);
        // backward W (M, N) and Y^T (K, N) for dX, X^T (K, M) and W (N, M) for dY
        size_t la = padlA(M), lb = padlB(N);
        size_t za = padlA(M) * padk(K), zb = padlB(N) * padk(K);
        size_t qa = pad256(M) * qlen(K), qb = padB(N) * qlen(K);
        size_t na = pad256(M), nb = padB(N);
        // CRT: per-modulus residues of each product (m x n, rows padded to 32)
        size_t out = (size_t)crt_residue_plane(M, N);
        if (bwd) {
            la = maxz(la, padlA(K));
            lb = maxz(lb, padlB(K));
            za = maxz(za, maxz(padlA(M) * padk(N), padlA(K) * padk(M)));
            zb = maxz(zb, maxz(padlB(K) * padk(N), padlB(N) * padk(M)));
            qa = maxz(qa, maxz(pad256(M) * qlen(N), pad256(K) * qlen(M)));
            qb = maxz(qb, maxz(padB(K) * qlen(N), padB(N) * qlen(M)));
            na = maxz(na, pad256(K));
            nb = maxz(nb, padB(K));
            out = maxz(out, maxz((size_t)crt_residue_plane(M, K), (size_t)crt_residue_plane(K, N)));
        }
        la = maxz(la, na);
        lb = maxz(lb, nb);
        L.mba = off; off += align_up(la * 8);
        L.mbb = off; off += align_up(lb * 8);
        L.ea = off; off += align_up(la * 4);
        L.eb = off; off += align_up(lb * 4);
        L.sxa = off; off += align_up(la * 8);
        L.sxb = off; off += align_up(lb * 8);
        L.psa = off; off += align_up((size_t)kColParts * la * 8);
        L.psb = off; off += align_up((size_t)kColParts * lb * 8);
        L.qa = off; off += align_up(qa);
        L.qb = off; off += align_up(qb);
        L.sa = off; off += align_up(planes * za * digit);
        L.sb = off; off += align_up(planes * zb * digit);
        if (is_crt(p)) {
            L.res = off;
            off += align_up(TCU_MAX_MODULI * out);
            L.need = off;
            off += align_up(out);
            L.exc = off;
            off += align_up((size_t)kExcThresholds * kExcCap * sizeof(int4));
        }
    } else {
        if (with_count_planes) {
            // the count's 0/1 planes (the mixed forms' magnitude planes hold
            // them there)
            L.qa = off; off += align_up(pad256(M) * qlen(K));
            L.qb = off; off += align_up(padB(N) * qlen(K));
        }
        // products with too few output tiles to fill the chip split their
        // contraction over workgroups (C = X Y; with backward also dX = dC
        // Y^T and dY = X^T dC), one partial product per k-chunk
        size_t sp = gemm_f64_split_bytes(M, N, K);
        if (bwd) sp = maxz(sp, maxz(gemm_f64_split_bytes(M, K, N), gemm_f64_split_bytes(K, N, M)));
        if (sp > 0) {
            L.gsplit = off;
            L.gsplit_bytes = sp;
            off += align_up(sp);
        }
    }
    L.total = off;
    return L;
}

// The FP64 form's split-contraction partials, or NULL (no product of the
// layout's shapes splits).
double *split_part(void *ws, const Layout &L) {
    return L.gsplit_bytes > 0 ? reinterpret_cast<double *>(static_cast<char *>(ws) + L.gsplit)
                              : nullptr;
}

bool ws_ok(const void *ws, size_t ws_bytes, size_t need) {
    return ws != nullptr && ((uintptr_t)ws % kAlign) == 0 && ws_bytes >= need;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// Scratch for window-by-window encodings: the workspace past the layout's
// end, when the caller sized it with the relations (tcu_workspace_bytes);
// a workspace without it encodes in one pass.
struct EncScratch {
    void *p = nullptr;
    size_t bytes = 0;
};

size_t enc_scratch_bytes(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                         int32_t N) {
    if (A == nullptr || B == nullptr) return 0;
    return std::max(encode_scratch_bytes(*A, M, K), encode_scratch_bytes(*B, K, N));
}

EncScratch enc_scratch(void *ws, size_t ws_bytes, const Layout &L, const tcu_relation *A,
                       const tcu_relation *B, int32_t M, int32_t K, int32_t N) {
    EncScratch e;
    const size_t need = enc_scratch_bytes(A, B, M, K, N);
    if (need > 0 && ws_bytes >= L.total + need) {
        e.p = static_cast<char *>(ws) + L.total;
        e.bytes = ws_bytes - L.total;
    }
    return e;
}

// One relation's encoding on stream s (the matrix zeroed, then the records
// placed; window by window for large matrices when there is scratch).
hipError_t encode_one(const tcu_relation &R, int which, int rows, int cols, double *Z,
                      StatusBlock *st, const EncScratch &sc, hipStream_t s) {
    return launch_encode_zeroed(R, which, rows, cols, Z, st, which, sc.p, sc.bytes, s);
}

// X (M x K) and Y (K x N) from the records; `count_only` encodes ones.
hipError_t encode_both(const tcu_relation &A, const tcu_relation &B, int32_t M, int32_t K,
                       int32_t N, double *X, double *Y, StatusBlock *st, bool count_only,
                       const EncScratch &sc, hipStream_t s) {
    tcu_relation a = A, b = B;
    if (count_only) { a.val = nullptr; b.val = nullptr; }
    // each matrix is zeroed right before its scatter, so its freshly written
    // lines are still in the caches when the random 8-byte stores land
    hipError_t e = encode_one(a, 0, M, K, X, st, sc, s);
    if (e == hipSuccess) e = encode_one(b, 1, K, N, Y, st, sc, s);
    return e;
}

// Mixed-form product C (m x n, ldc) = opA * opB with contraction length k.
// opA's lines are its m rows: Za with axis_a (0: Za is m x k, rows are
// lines; 1: Za is k x m, columns are lines); likewise opB's n lines from Zb
// with axis_b (0: Zb is n x k; 1: Zb is k x n).
struct SplitOperand {
    const double *Z;
    int rows, cols;
    int64_t ld;
    int axis;
};

// Plan of one mixed-form product: the slice count S (or modulus count, with
// the truncation width `bits`; S = 0: no certified plan, the product runs in
// FP64), the padded contraction length and the padded line counts.
struct MixedPlan {
    int S = 0, bits = 0, len_pad = 0, la = 0, lb = 0;
    uint32_t need = 0;  // the certificate's need in this form
    uint32_t exc = 0;   // residue form: cells needing more than `bits`, recomputed alone
    int exc_last = -1;  // the last list segment they fill
};

// Step a0 for one operand: line maxima and sums of |z|, then the magnitude
// plane and normalised sums of the certificate.
hipError_t certify_prepare(const SplitOperand &o, bool second, void *ws, const Layout &L,
                           StatusBlock *st, hipStream_t s) {
    auto *mb = at<unsigned long long>(ws, second ? L.mbb : L.mba);
    double *ps = at<double>(ws, second ? L.psb : L.psa);
    const int lines = o.axis == 0 ? o.rows : o.cols, len = o.axis == 0 ? o.cols : o.rows;
    hipError_t e = launch_line_max(o.Z, o.rows, o.cols, o.ld, o.axis, mb, ps, st, s);
    if (e != hipSuccess) return e;
    return launch_mag_plane(o.Z, o.rows, o.cols, o.ld, o.axis, mb, ps,
                            at<double>(ws, second ? L.sxb : L.sxa),
                            second ? &st->umax_b : &st->umax_a,
                            at<int8_t>(ws, second ? L.qb : L.qa),
                            (int)(second ? padB(lines) : pad256(lines)),
                            (int)qlen(len), s);
}

// Exceptions of the residue form.  The certificate's plan truncates every
// line to the widest need over all cells.  When a few cells need more than
// the rest, a narrower width b can take fewer moduli: the cells needing more
// than b (and any the certificate cannot bound) are then recomputed one by
// one as compensated FP64 dot products after the reconstruction, which
// keeps every cell within tol (|X||Y|)[g,h].  The candidate widths are the
// widest ones at which the modulus count drops, level by level below the
// certificate's plan; one scan of the need plane lists the cells above each
// of them (in segments, so that a level whose cells fit the list is usable
// even when a deeper one overflows), and the plan takes the level with the
// least estimated time.

// moduli for width b (0: none suffice)
int crt_moduli_for(int32_t k, double tol, int b, double u) {
    int32_t bits = 0;
    const int r = mixed_plan(TCU_PREC_CRT_I8, k, tol, (uint32_t)b, u, &bits);
    return r > 0 ? r : 0;
}

// Estimated seconds of the residue products (L moduli) of an m x n x k
// product and of the FP64 product that replaces a plan without moduli
// (L = 0); of the scan, which reads the need plane and synchronises once
// more; and of recomputing cells alone (row and column read with a 64-byte
// sector per element when strided).
double crt_seconds(int L, int m, int n, int k) {
    const double mnk = 2.0 * m * n * (double)k;
    return L > 0 ? L * mnk / 2.5e15 : mnk / 6.0e13;
}
double scan_seconds(int m, int n) { return (double)((m + 31) / 32 * 32) * n / 2.0e12 + 2e-5; }
double fixup_seconds(uint32_t cells, int k) {
    return cells == 0 ? 0.0 : cells * 2.0 * k * 64.0 / 1.0e12 + 1e-5;
}

// Candidate widths, widest first, and their modulus counts: for each count
// below the certificate's plan (L0 moduli; 0: no plan), the widest width
// that takes it, from the widest allowed down (below the largest need, or
// with cells the certificate cannot bound or wider than 53 bits, at most
// the largest bounded need within 53).
struct ExcLevels {
    int n = 0;
    int b[kExcThresholds] = {}, L[kExcThresholds] = {};
};

ExcLevels exception_levels(int32_t k, double tol, uint32_t need_all, uint32_t need_cert, double u,
                           int L0) {
    ExcLevels lv;
    int hi;
    if (need_all < kNeedUncertified && need_all <= 53)
        hi = (int)need_all - 1;
    else
        hi = std::max(1, std::min((int)need_cert, 53));
    int cur = L0;
    for (int b = hi; b >= 1 && lv.n < kExcThresholds; --b) {
        const int Lb = crt_moduli_for(k, tol, b, u);
        if (Lb > 0 && (cur == 0 || Lb < cur)) {
            lv.b[lv.n] = b;
            lv.L[lv.n] = Lb;
            ++lv.n;
            cur = Lb;
        }
    }
    return lv;
}

// Whether the scan pays: the first level's saving against twice its cost.
// When even the smallest nonzero need of a bounded cell exceeds the first
// level's width, every such cell would be an exception: no scan.  (With no
// bounded cell of nonzero need, need_min stays 255 and only the cells the
// certificate cannot bound can be exceptions.)
bool exception_scan_pays(int m, int n, int k, int L0, const ExcLevels &lv, uint32_t need_min) {
    if (lv.n == 0) return false;
    if (need_min < kNeedUncertified && need_min > (uint32_t)lv.b[0]) return false;
    const double gain = crt_seconds(L0, m, n, k) - crt_seconds(lv.L[0], m, n, k);
    return gain > 2.0 * scan_seconds(m, n);
}

struct ExcPlan {
    int L = 0, bits = 0, last = -1;  // L = 0: keep the certificate's plan
    uint32_t exc = 0;
};

// After the scan (seg[j]: cells listed in segment j, above cap: overflowed):
// the level with the least estimated time, if it beats the certificate's
// plan; a level needs every segment up to its own complete.
ExcPlan exception_plan(int m, int n, int32_t k, int L0, const ExcLevels &lv,
                       const uint32_t *seg) {
    ExcPlan best;
    double best_t = crt_seconds(L0, m, n, k);
    uint32_t cells = 0;
    for (int j = 0; j < lv.n; ++j) {
        if (seg[j] > kExcCap) break;
        cells += seg[j];
        const double t = crt_seconds(lv.L[j], m, n, k) + fixup_seconds(cells, k);
        if (t < best_t) {
            best_t = t;
            best.L = lv.L[j];
            best.bits = lv.b[j];
            best.last = j;
            best.exc = cells;
        }
    }
    return best;
}

// The certificate of a product whose operands went through certify_prepare,
// then the plan.  Reads the certificate back: SYNCHRONISES the stream (and
// once more when it scans for exceptions).
hipError_t certify_and_plan(int m, int n, int k, tcu_precision p, double tol, void *ws,
                            const Layout &L, StatusBlock *st, MixedPlan *mp, hipStream_t s) {
    tol = tol_or_default(tol);
    CertArgs ca{};
    ca.sx = at<double>(ws, L.sxa);
    ca.sy = at<double>(ws, L.sxb);
    // the residue form's reconstruction rounds once, the digit forms'
    // combination once per FP64 addition; the factor keeps the comparisons
    // on the safe side of their own roundings
    ca.tcrt = (tol - 0x1p-52) * (1.0 - 0x1p-40);
    ca.kterm = 16384.0 * (double)k;
    for (int S = 1; S <= TCU_MAX_SLICES; ++S)
        ca.tdig[S] = is_crt(p) ? 0.0
                               : (tol - (double)digit_adds(S, p == TCU_PREC_SPLIT_BF16, k) *
                                            0x1p-52) * (1.0 - 0x1p-40);
    ca.need_bits = &st->need_bits;
    ca.need_slices = &st->need_slices;
    if (is_crt(p)) {
        ca.need_plane = at<uint8_t>(ws, L.need);
        ca.need_cert = &st->need_cert;
        ca.need_min = &st->need_min;
    }
    hipError_t e = launch_certify(m, n, k, at<int8_t>(ws, L.qa), (int)pad256(m),
                                  at<int8_t>(ws, L.qb), (int)padB(n), (int)qlen(k), ca,
                                  !is_crt(p), s);
    if (e != hipSuccess) return e;
    StatusBlock host;
    e = hipMemcpyAsync(&host, st, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    double ua, ub;
    memcpy(&ua, &host.umax_a, sizeof(ua));
    memcpy(&ub, &host.umax_b, sizeof(ub));
    int32_t bits = 0;
    int r = TCU_ERR_NONFINITE;
    if (!(host.flags & kFlagNonFinite))
        r = mixed_plan(p, k, tol, is_crt(p) ? host.need_bits : host.need_slices,
                       std::min(ua, ub), &bits);
    *mp = MixedPlan{};
    mp->need = is_crt(p) ? host.need_bits : host.need_slices;
    if (is_crt(p) && !(host.flags & kFlagNonFinite)) {
        // a narrower width whose few wider-need cells are recomputed alone
        const int L0 = r > 0 ? r : 0;
        const ExcLevels lv = exception_levels(k, tol, host.need_bits, host.need_cert,
                                              std::min(ua, ub), L0);
        if (exception_scan_pays(m, n, k, L0, lv, host.need_min)) {
            ExcThresholds thr;
            for (int j = 0; j < kExcThresholds; ++j)
                thr.t[j] = j < lv.n ? (uint32_t)lv.b[j] : 255u;
            e = launch_need_scan(at<uint8_t>(ws, L.need), m, n, thr, at<int4>(ws, L.exc),
                                 kExcCap, st, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&host, st, sizeof(host), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            const ExcPlan xp = exception_plan(m, n, k, L0, lv, host.exc_seg);
            if (xp.L > 0) {
                r = xp.L;
                bits = xp.bits;
                mp->exc = xp.exc;
                mp->exc_last = xp.last;
            }
        }
    }
    if (r > 0) {
        mp->S = r;
        mp->bits = bits;
        if (is_crt(p)) {
            mp->len_pad = (int)qlen(k);
            mp->la = (int)pad256(m);
            mp->lb = (int)padB(n);
        } else {
            mp->len_pad = (int)pad64(k);
            mp->la = (int)pad128(m);
            mp->lb = (int)pad128(n);
        }
    }
    return hipSuccess;
}

// Digit slices or residues of one operand under the plan (its line maxima
// are in place from certify_prepare), into the workspace buffers of side A
// (second = false) or side B.
hipError_t mixed_split(const SplitOperand &o, bool second, const MixedPlan &mp, tcu_precision p,
                       void *ws, const Layout &L, hipStream_t s) {
    const auto *mb = at<unsigned long long>(ws, second ? L.mbb : L.mba);
    int *ex = at<int>(ws, second ? L.eb : L.ea);
    const int lines = second ? mp.lb : mp.la;
    if (is_crt(p))
        return launch_crt_split(o.Z, o.rows, o.cols, o.ld, o.axis, mb, mp.S, mp.bits,
                                at<int8_t>(ws, second ? L.sb : L.sa), lines, mp.len_pad, ex, s);
    return launch_split(o.Z, o.rows, o.cols, o.ld, o.axis, mb, mp.S, p == TCU_PREC_SPLIT_BF16,
                        at<char>(ws, second ? L.sb : L.sa), lines, mp.len_pad, ex, s);
}

// The narrow products of both prepared operands and their FP64 combination.
hipError_t mixed_multiply(int m, int n, int k, const MixedPlan &mp, tcu_precision p, void *ws,
                          const Layout &L, double *C, int64_t ldc, hipStream_t s) {
    const int *ea = at<int>(ws, L.ea), *eb = at<int>(ws, L.eb);
    if (is_crt(p))
        return launch_gemm_crt(m, n, k, mp.S, mp.bits, at<int8_t>(ws, L.sa), mp.la,
                               at<int8_t>(ws, L.sb), mp.lb, mp.len_pad, at<int8_t>(ws, L.res), ea,
                               eb, C, ldc, 0, s);
    return launch_gemm_split(m, n, k, mp.S, p == TCU_PREC_SPLIT_BF16, at<char>(ws, L.sa), mp.la,
                             at<char>(ws, L.sb), mp.lb, mp.len_pad, ea, eb, C, ldc, s);
}

// The rest of a product once both operands went through certify_prepare:
// certificate and plan, then the narrow products, or the FP64 product of
// the same operands when no plan is certified (recorded in the status
// block with the plan).
hipError_t finish_product(const SplitOperand &a, const SplitOperand &b, int m, int n, int k,
                          tcu_precision p, double tol, void *ws, const Layout &L, StatusBlock *st,
                          double *C, int64_t ldc, hipStream_t s) {
    MixedPlan mp;
    hipError_t e = certify_and_plan(m, n, k, p, tol, ws, L, st, &mp, s);
    if (e != hipSuccess) return e;
    if (mp.S == 0) {
        e = launch_gemm_f64(a.axis, b.axis == 0 ? 1 : 0, m, n, k, a.Z, a.ld, b.Z, b.ld, C, ldc, s);
        if (e == hipSuccess) e = launch_set_plan(st, 0, 0, mp.need, true, s);
        return e;
    }
    e = mixed_split(a, false, mp, p, ws, L, s);
    if (e == hipSuccess) e = mixed_split(b, true, mp, p, ws, L, s);
    if (e == hipSuccess) e = mixed_multiply(m, n, k, mp, p, ws, L, C, ldc, s);
    if (e == hipSuccess && mp.exc > 0)
        e = launch_exception_fixup(at<int4>(ws, L.exc), st, kExcCap, mp.exc_last, k, a.Z, a.ld,
                                   a.axis, b.Z, b.ld, b.axis, C, ldc, s);
    if (e == hipSuccess)
        e = launch_set_plan(st, (uint32_t)mp.S, (uint32_t)mp.bits, mp.need, false, s, mp.exc);
    return e;
}

// One whole mixed-form product of two dense operands.
hipError_t mixed_product(const SplitOperand &a, const SplitOperand &b, int m, int n, int k,
                         tcu_precision p, double tol, void *ws, const Layout &L, StatusBlock *st,
                         double *C, int64_t ldc, hipStream_t s) {
    hipError_t e = launch_reset_plan(st, s);
    if (e == hipSuccess) e = certify_prepare(a, false, ws, L, st, s);
    if (e == hipSuccess) e = certify_prepare(b, true, ws, L, st, s);
    if (e == hipSuccess) e = finish_product(a, b, m, n, k, p, tol, ws, L, st, C, ldc, s);
    return e;
}

// The adjoint's second stream: one non-blocking stream (default priority) per
// device, created on first use and kept for the life of the process.  Work
// on it is ordered against the caller's stream by events only, so a call
// stays stream-ordered with respect to the caller's stream.
hipError_t side_stream(hipStream_t *out) {
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (streams[dev] == nullptr) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            streams[dev] = nullptr;
            return e;
        }
    }
    *out = streams[dev];
    return hipSuccess;
}

// Events of one call, destroyed when the call returns (the runtime
// keeps a recorded event alive until the work it marks has run).  Once work
// has been forked to the internal stream, leaving the call without the
// normal join (an early error return) still orders the caller's stream after
// everything queued there, since that work writes the caller's buffers.
struct CallEvents {
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipStream_t side = nullptr, caller = nullptr;
    bool joined = false;
    hipError_t create() {
        for (hipEvent_t &e : ev) {
            const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    void forked(hipStream_t s, hipStream_t c) {
        side = s;
        caller = c;
    }
    // the caller's stream waits for `e`, recorded after the side's last work
    hipError_t join(hipEvent_t e) {
        joined = true;
        return hipStreamWaitEvent(caller, e, 0);
    }
    ~CallEvents() {
        if (side != nullptr && !joined && ev[2] != nullptr &&
            hipEventRecord(ev[2], side) == hipSuccess)
            (void)hipStreamWaitEvent(caller, ev[2], 0);
        for (hipEvent_t e : ev)
            if (e != nullptr) (void)hipEventDestroy(e);
    }
};

}  // namespace

LaunchTrace &tcu::launch_trace() {
    static thread_local LaunchTrace t;
    return t;
}

extern "C" {

tcu_status tcu_trace_launches(tcu_launch_record *records, int32_t capacity, int32_t *count) {
    LaunchTrace &t = launch_trace();
    if (count == nullptr) {
        t = LaunchTrace{};
        return TCU_OK;
    }
    if (capacity < 0 || (capacity > 0 && records == nullptr)) return TCU_ERR_ARG;
    *count = 0;
    t.rec = records;
    t.cap = capacity;
    t.count = count;
    return TCU_OK;
}

size_t tcu_workspace_bytes(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                           int32_t N, tcu_precision p, int flags) {
    if (!shapes_ok(M, K, N)) return 0;
    if (!precision_ok(p)) return 0;
    return plan_layout(M, K, N, p, flags, count_planes(A, B, flags)).total +
           enc_scratch_bytes(A, B, M, K, N);
}

int tcu_mixed_plan(tcu_precision p, int32_t k, double tol, uint32_t need, double u,
                   int32_t *bits) {
    return mixed_plan(p, k, tol, need, u, bits);
}

tcu_status tcu_split(const double *Z, int32_t rows, int32_t cols, int64_t ld, int axis,
                     tcu_precision p, int32_t S, void *slices, int32_t lines_pad,
                     int32_t len_pad, int32_t *exps, void *ws, size_t ws_bytes,
                     hipStream_t stream) {
    if (Z == nullptr || slices == nullptr || exps == nullptr) return TCU_ERR_ARG;
    if (rows < 1 || cols < 1 || ld < cols || (axis != 0 && axis != 1)) return TCU_ERR_ARG;
    if (!is_split(p) || is_crt(p) || S < 1 || S > TCU_MAX_SLICES) return TCU_ERR_ARG;
    const int lines = axis == 0 ? rows : cols, len = axis == 0 ? cols : rows;
    if (lines_pad < lines || lines_pad % 128 || len_pad < len || len_pad % 64) return TCU_ERR_ARG;
    if (!ws_ok(ws, ws_bytes, sizeof(StatusBlock) + (size_t)lines_pad * 8)) return TCU_ERR_WORKSPACE;
    StatusBlock *st = at<StatusBlock>(ws, 0);
    auto *mb = at<unsigned long long>(ws, sizeof(StatusBlock));
    TCU_TRY(launch_clear_status(st, stream, (uint32_t)S));
    TCU_TRY(launch_line_max(Z, rows, cols, ld, axis, mb, nullptr, st, stream));
    TCU_TRY(launch_split(Z, rows, cols, ld, axis, mb, S, p == TCU_PREC_SPLIT_BF16, slices,
                         lines_pad, len_pad, exps, stream));
    return TCU_OK;
}

tcu_status tcu_encode(const tcu_relation *R, int transpose, int32_t rows, int32_t cols,
                      double *out, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!relation_ok(R) || rows < 1 || cols < 1 || out == nullptr) return TCU_ERR_ARG;
    if (transpose != 0 && transpose != 1) return TCU_ERR_ARG;
    if (!ws_ok(ws, ws_bytes, sizeof(StatusBlock))) return TCU_ERR_WORKSPACE;
    StatusBlock *st = at<StatusBlock>(ws, 0);
    TCU_TRY(launch_clear_status(st, stream));
    // the workspace past the status block, if large enough, lets a large
    // matrix be filled window by window
    TCU_TRY(launch_encode_zeroed(*R, transpose, rows, cols, out, st, 0,
                                 static_cast<char *>(ws) + sizeof(StatusBlock),
                                 ws_bytes - sizeof(StatusBlock), stream));
    return TCU_OK;
}

size_t tcu_encode_workspace_bytes(const tcu_relation *R, int32_t rows, int32_t cols) {
    if (!relation_ok(R) || rows < 1 || cols < 1) return 0;
    return sizeof(StatusBlock) + encode_scratch_bytes(*R, rows, cols);
}

tcu_status tcu_gemm_f64(int trans_a, int trans_b, int32_t m, int32_t n, int32_t k,
                        const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                        int64_t ldc, hipStream_t stream) {
    if ((trans_a != 0 && trans_a != 1) || (trans_b != 0 && trans_b != 1)) return TCU_ERR_ARG;
    if (m < 0 || n < 0 || k < 0) return TCU_ERR_ARG;
    if (m == 0 || n == 0) return TCU_OK;
    if (C == nullptr || ldc < n) return TCU_ERR_ARG;
    if (k > 0) {
        if (A == nullptr || B == nullptr) return TCU_ERR_ARG;
        if (lda < (trans_a ? m : k) || ldb < (trans_b ? k : n)) return TCU_ERR_ARG;
    }
    return hip_status(launch_gemm_f64(trans_a, trans_b, m, n, k, A, lda, B, ldb, C, ldc, stream));
}

size_t tcu_gemm_f64_workspace_bytes(int32_t m, int32_t n, int32_t k) {
    if (m < 1 || n < 1 || k < 1) return 0;
    return gemm_f64_split_bytes(m, n, k);
}

tcu_status tcu_gemm_f64_ws(int trans_a, int trans_b, int32_t m, int32_t n, int32_t k,
                           const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                           int64_t ldc, void *ws, size_t ws_bytes, hipStream_t stream) {
    if ((trans_a != 0 && trans_a != 1) || (trans_b != 0 && trans_b != 1)) return TCU_ERR_ARG;
    if (m < 0 || n < 0 || k < 0) return TCU_ERR_ARG;
    if (m == 0 || n == 0) return TCU_OK;
    if (C == nullptr || ldc < n) return TCU_ERR_ARG;
    if (k > 0) {
        if (A == nullptr || B == nullptr) return TCU_ERR_ARG;
        if (lda < (trans_a ? m : k) || ldb < (trans_b ? k : n)) return TCU_ERR_ARG;
    }
    const size_t need = k > 0 ? gemm_f64_split_bytes(m, n, k) : 0;
    if (need > 0 && !ws_ok(ws, ws_bytes, need)) return TCU_ERR_WORKSPACE;
    return hip_status(launch_gemm_f64_split(trans_a, trans_b, m, n, k, A, lda, B, ldb, C, ldc,
                                            need > 0 ? static_cast<double *>(ws) : nullptr,
                                            stream));
}

tcu_status tcu_join_agg_fwd(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, tcu_precision p, double tol, double *C, int32_t *count,
                            void *ws, size_t ws_bytes, hipStream_t stream) {
    return join_agg_fwd_ws(A, B, M, K, N, p, tol, C, count, ws, ws_bytes, stream);
}

}  // extern "C"

// The forward on a given workspace: the body of tcu_join_agg_fwd, shared with
// tcu_join_agg_fwd_noalloc (whose workspace is the library's own device array).
tcu_status tcu::join_agg_fwd_ws(const tcu_relation *A, const tcu_relation *B, int32_t M,
                                int32_t K, int32_t N, tcu_precision p, double tol, double *C,
                                int32_t *count, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!relation_ok(A) || !relation_ok(B) || !shapes_ok(M, K, N) || C == nullptr)
        return TCU_ERR_ARG;
    if (!precision_ok(p)) return TCU_ERR_ARG;
    if (is_split(p) && !mixed_shape_ok(p, K, tol)) return TCU_ERR_INFEASIBLE;
    const bool planes = count != nullptr && count_planes(A, B, TCU_WS_COUNT);
    const Layout L = plan_layout(M, K, N, p, 0, planes);
    if (!ws_ok(ws, ws_bytes, L.total)) return TCU_ERR_WORKSPACE;
    StatusBlock *st = at<StatusBlock>(ws, 0);
    double *X = at<double>(ws, L.x), *Y = at<double>(ws, L.y);
    const EncScratch sc = enc_scratch(ws, ws_bytes, L, A, B, M, K, N);

    TCU_TRY(launch_clear_status(st, stream));
    if (planes) {
        // exact pair counts, Section 3.1's 0/1 encodings (unique cells): one
        // int8 product with exact int32 sums (K < 2^31)
        int8_t *qa = at<int8_t>(ws, L.qa), *qb = at<int8_t>(ws, L.qb);
        TCU_TRY(launch_count_planes(*A, M, K, qa, (int)pad256(M), (int)qlen(K), stream));
        TCU_TRY(launch_count_planes(*B, N, K, qb, (int)padB(N), (int)qlen(K), stream));
        TCU_TRY(launch_count_product(M, N, K, qa, (int)pad256(M), qb, (int)padB(N),
                                     (int)qlen(K), count, N, stream));
    } else if (count != nullptr) {
        // the multiplicity encodings of Section 3.1, multiplied in FP64 (every
        // partial sum is a non-negative integer no larger than the count, so a
        // count below 2^53 is exact), C as scratch; counts beyond int32 are
        // saturated and flagged
        TCU_TRY(encode_both(*A, *B, M, K, N, X, Y, nullptr, true, sc, stream));
        TCU_TRY(launch_gemm_f64_split(0, 0, M, N, K, X, K, Y, N, C, N, split_part(ws, L), stream));
        TCU_TRY(launch_f64_to_i32(C, count, (size_t)M * N, st, stream));
    }
    if (!is_split(p)) {
        TCU_TRY(encode_both(*A, *B, M, K, N, X, Y, st, false, sc, stream));
        TCU_TRY(launch_gemm_f64_split(0, 0, M, N, K, X, K, Y, N, C, N, split_part(ws, L), stream));
        return TCU_OK;
    }
    // Mixed forms: each operand is encoded and at once reduced to its line
    // statistics and magnitude plane, which read it while it is still in the
    // caches; then the other operand, the certificate and the plan.
    // X: M lines (rows) of length K; Y: N lines (columns) of length K
    const SplitOperand a{X, M, K, K, 0}, b{Y, K, N, N, 1};
    TCU_TRY(launch_reset_plan(st, stream));
    TCU_TRY(encode_one(*A, 0, M, K, X, st, sc, stream));
    TCU_TRY(certify_prepare(a, false, ws, L, st, stream));
    TCU_TRY(encode_one(*B, 1, K, N, Y, st, sc, stream));
    TCU_TRY(certify_prepare(b, true, ws, L, st, stream));
    TCU_TRY(finish_product(a, b, M, N, K, p, tol, ws, L, st, C, N, stream));
    return TCU_OK;
}

size_t tcu::join_agg_fwd_ws_bytes(const tcu_relation *A, const tcu_relation *B, int32_t M,
                                  int32_t K, int32_t N, tcu_precision p, bool with_count) {
    if (!shapes_ok(M, K, N) || !precision_ok(p)) return 0;
    return plan_layout(M, K, N, p, 0, with_count && count_planes(A, B, TCU_WS_COUNT)).total;
}

extern "C" {

tcu_status tcu_join_agg_bwd(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, tcu_precision p, double tol, const double *dC,
                            double *dA_val, double *dB_val, int flags, void *ws,
                            size_t ws_bytes, hipStream_t stream) {
    if (!relation_ok(A) || !relation_ok(B) || !shapes_ok(M, K, N) || dC == nullptr)
        return TCU_ERR_ARG;
    if ((flags & ~TCU_BWD_SAVED_ENCODINGS) != 0) return TCU_ERR_ARG;
    if (!precision_ok(p)) return TCU_ERR_ARG;
    // dX contracts over h (length N), dY over g (length M)
    if (is_split(p) && (!mixed_shape_ok(p, N, tol) || !mixed_shape_ok(p, M, tol)))
        return TCU_ERR_INFEASIBLE;
    const bool mixed = is_split(p);
    const Layout L = plan_layout(M, K, N, p, TCU_WS_BACKWARD);
    if (!ws_ok(ws, ws_bytes, L.total)) return TCU_ERR_WORKSPACE;
    StatusBlock *st = at<StatusBlock>(ws, 0);
    double *X = at<double>(ws, L.x), *Y = at<double>(ws, L.y);
    double *G = at<double>(ws, L.g), *G2 = at<double>(ws, L.g2);
    // Y's re-encoding ends (stream order) before X's starts on the side
    // stream, so the two share the scratch
    const EncScratch sc = enc_scratch(ws, ws_bytes, L, A, B, M, K, N);

    if (dA_val == nullptr && dB_val == nullptr) return TCU_OK;
    const bool saved = (flags & TCU_BWD_SAVED_ENCODINGS) != 0;
    // With both gradients, the gather of dA (memory-bound) and, when the
    // encodings are rebuilt, the encoding of X run on a second stream beside
    // the matrix products on the caller's stream:
    //   caller: [encode Y] fork  dX = dC Y^T  ev_dx  ...wait ev_x  dY = X^T dC  wait ev_a  gather dB
    //   side:        wait fork  [encode X] ev_x  wait ev_dx  gather dA  ev_a
    // (the FP64 dY product may be cut in two, its first part's dB gather
    // joining the side stream; see below).
    // dX and dY live in separate buffers (G, G2), so nothing the two streams
    // run at the same time touches the same memory.
    const bool both = dA_val != nullptr && dB_val != nullptr;
    hipStream_t side = nullptr;
    CallEvents evs;
    if (both) {
        TCU_TRY(side_stream(&side));
        TCU_TRY(evs.create());
    }
    hipEvent_t ev_fork = evs.ev[0], ev_x = evs.ev[1], ev_a = evs.ev[2];

    if (!saved) {
        // activation checkpointing: the encodings are rebuilt from the records
        TCU_TRY(launch_clear_status(st, stream));
        TCU_TRY(encode_one(*B, 1, K, N, Y, st, sc, stream));
        if (both) {
            TCU_TRY(hipEventRecord(ev_fork, stream));
            TCU_TRY(hipStreamWaitEvent(side, ev_fork, 0));
            evs.forked(side, stream);
            TCU_TRY(encode_one(*A, 0, M, K, X, st, sc, side));
            TCU_TRY(hipEventRecord(ev_x, side));
        } else {
            TCU_TRY(encode_one(*A, 0, M, K, X, st, sc, stream));
        }
    }
    if (dA_val != nullptr) {
        // dX = dC * Y^T (M x K), then dA.val[i] = dX[g_i, k_i]
        if (!mixed) {
            TCU_TRY(launch_gemm_f64_split(0, 1, M, K, N, dC, N, Y, N, G, K, split_part(ws, L),
                                          stream));
        } else {
            // dC: M lines (rows) of length N; Y^T: K lines = rows of Y, length N
            const SplitOperand a{dC, M, N, N, 0}, b{Y, K, N, N, 0};
            TCU_TRY(mixed_product(a, b, M, K, N, p, tol, ws, L, st, G, K, stream));
        }
        if (both) {
            // ev_fork is free again once the side stream has waited for it
            TCU_TRY(hipEventRecord(ev_fork, stream));
            TCU_TRY(hipStreamWaitEvent(side, ev_fork, 0));
            evs.forked(side, stream);
            TCU_TRY(launch_gather(*A, 0, M, K, G, dA_val, side));
            TCU_TRY(hipEventRecord(ev_a, side));
        } else {
            TCU_TRY(launch_gather(*A, 0, M, K, G, dA_val, stream));
        }
    }
    if (dB_val != nullptr) {
        if (both && !saved) TCU_TRY(hipStreamWaitEvent(stream, ev_x, 0));  // X is encoded
        // dY = X^T * dC (K x N), then dB.val[j] = dY[k_j, h_j]
        // With both gradients, the FP64 product is cut into two row blocks
        // when that costs no extra round of workgroups: the dB gather of the
        // first block's records runs on the side stream beside the second
        // block's product, and only the second block's gather stays behind.
        const int k1 = (both && !mixed) ? gemm_f64_row_cut(K, N) : 0;
        if (k1 > 0) {
            TCU_TRY(launch_gemm_f64(1, 0, k1, N, M, X, K, dC, N, G2, N, stream));
            TCU_TRY(hipEventRecord(ev_fork, stream));
            TCU_TRY(hipStreamWaitEvent(side, ev_fork, 0));
            TCU_TRY(launch_gather(*B, 1, K, N, G2, dB_val, side, 0, k1));
            TCU_TRY(hipEventRecord(ev_a, side));
            TCU_TRY(launch_gemm_f64(1, 0, K - k1, N, M, X + k1, K, dC, N, G2 + (size_t)k1 * N, N,
                                    stream));
        } else if (!mixed) {
            TCU_TRY(launch_gemm_f64_split(1, 0, K, N, M, X, K, dC, N, G2, N, split_part(ws, L),
                                          stream));
        } else {
            // X^T: K lines = columns of X, length M; dC: N lines = columns, length M
            const SplitOperand a{X, M, K, K, 1}, b{dC, M, N, N, 1};
            TCU_TRY(mixed_product(a, b, K, N, M, p, tol, ws, L, st, G2, N, stream));
        }
        TCU_TRY(launch_gather(*B, 1, K, N, G2, dB_val, stream, k1, K));
        if (both) TCU_TRY(evs.join(ev_a));  // the side's gathers are done
    }
    return TCU_OK;
}

size_t tcu_mfma_peak_out_bytes(void) { return mfma_peak_out_bytes(); }

double tcu_mfma_peak_ops(int kind, int32_t iters) {
    if (kind < 0 || kind > 2 || iters < 1) return 0.0;
    return mfma_peak_ops(kind, iters);
}

tcu_status tcu_mfma_peak(int kind, int32_t iters, void *out, hipStream_t stream) {
    if (kind < 0 || kind > 2 || iters < 1 || out == nullptr) return TCU_ERR_ARG;
    return hip_status(launch_mfma_peak(kind, iters, out, stream));
}

size_t tcu_dict_workspace_bytes(int64_t n) {
    if (n < 0 || n > 0x7fffffffLL) return 0;
    return dict_workspace_bytes(n);
}

tcu_status tcu_dict_encode(const int64_t *a, int64_t n_a, const int64_t *b, int64_t n_b,
                           int32_t *codes_a, int32_t *codes_b, int64_t *dict, int64_t *k,
                           void *ws, size_t ws_bytes, hipStream_t stream) {
    if (n_a < 0 || n_b < 0 || n_a + n_b > 0x7fffffffLL || k == nullptr) return TCU_ERR_ARG;
    if ((n_a > 0 && (a == nullptr || codes_a == nullptr)) ||
        (n_b > 0 && (b == nullptr || codes_b == nullptr)) || (n_a + n_b > 0 && dict == nullptr))
        return TCU_ERR_ARG;
    if (!ws_ok(ws, ws_bytes, dict_workspace_bytes(n_a + n_b))) return TCU_ERR_WORKSPACE;
    return hip_status(run_dict_encode(reinterpret_cast<const long long *>(a), n_a,
                                      reinterpret_cast<const long long *>(b), n_b, codes_a,
                                      codes_b, reinterpret_cast<long long *>(dict), k, ws,
                                      stream));
}

size_t tcu_join_agg_row_workspace_bytes(int32_t K, int32_t N) {
    if (K < 1 || N < 1) return 0;
    return row_workspace_bytes(K, N);
}

tcu_status tcu_join_agg_row(const tcu_relation *A, const tcu_relation *B, int32_t K, int32_t N,
                            double *c, uint64_t *count, void *ws, size_t ws_bytes,
                            hipStream_t stream) {
    if (!relation_ok(A) || !relation_ok(B) || K < 1 || N < 1 || c == nullptr) return TCU_ERR_ARG;
    if (!ws_ok(ws, ws_bytes, row_workspace_bytes(K, N))) return TCU_ERR_WORKSPACE;
    return hip_status(run_join_agg_row(*A, *B, K, N, c,
                                       reinterpret_cast<unsigned long long *>(count), ws,
                                       stream));
}

size_t tcu_join_agg_bsr_workspace_bytes(const tcu_relation *A, const tcu_relation *B,
                                        int32_t M, int32_t K, int32_t N) {
    if (!relation_ok(A) || !relation_ok(B) || !shapes_ok(M, K, N)) return 0;
    return bsr_workspace_bytes(A->n, B->n, M, K, N);
}

tcu_status tcu_join_agg_bsr(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, double *C, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!relation_ok(A) || !relation_ok(B) || !shapes_ok(M, K, N) || C == nullptr)
        return TCU_ERR_ARG;
    if (A->n > 0x7fffffffLL || B->n > 0x7fffffffLL) return TCU_ERR_ARG;
    if (!ws_ok(ws, ws_bytes, bsr_workspace_bytes(A->n, B->n, M, K, N))) return TCU_ERR_WORKSPACE;
    return hip_status(run_join_agg_bsr(*A, *B, M, K, N, C, ws, stream));
}

int tcu_block_sparse_preferred(const tcu_relation *A, const tcu_relation *B, int32_t M,
                               int32_t K, int32_t N) {
    if (!relation_ok(A) || !relation_ok(B) || !shapes_ok(M, K, N)) return TCU_ERR_ARG;
    const double tm = (M + 15) / 16, tk = (K + 15) / 16, tn = (N + 15) / 16;
    const double dense_ms = 2.0 * M * (double)N * K / 70e12 * 1e3 +
                            16.0 * ((double)M * K + (double)K * N) / 3e12 * 1e3;
    const double ta = std::min((double)A->n, tm * tk), tb = std::min((double)B->n, tk * tn);
    const double meetings = ta * tb / tk;
    const double bsr_ms = 0.62 + 1.7e-6 * tm * tn + 1.4e-7 * meetings;
    return bsr_ms < dense_ms ? 1 : 0;
}

size_t tcu_nonzero_workspace_bytes(int64_t rows, int64_t cols) {
    if (rows < 0 || cols < 0 || rows > 0x7fffffffLL || cols > 0x7fffffffLL) return 0;
    return nonzero_workspace_bytes(rows, cols);
}

tcu_status tcu_nonzero(const double *M, int64_t rows, int64_t cols, int64_t ld, int32_t *out_row,
                       int32_t *out_col, const int32_t *col_map, int32_t *out_key,
                       int64_t capacity, int64_t *count, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
    if (rows < 0 || cols < 0 || rows > 0x7fffffffLL || cols > 0x7fffffffLL || ld < cols ||
        capacity < 0 || count == nullptr)
        return TCU_ERR_ARG;
    if (rows * cols > 0 && M == nullptr) return TCU_ERR_ARG;
    if (capacity > 0 && (out_row == nullptr || out_col == nullptr)) return TCU_ERR_ARG;
    if ((col_map == nullptr) != (out_key == nullptr)) return TCU_ERR_ARG;
    if (!ws_ok(ws, ws_bytes, nonzero_workspace_bytes(rows, cols))) return TCU_ERR_WORKSPACE;
    return hip_status(run_nonzero(M, rows, cols, ld, out_row, out_col, col_map, out_key, capacity,
                                  count, ws, stream));
}

tcu_status tcu_gemm_f64_host(int32_t m, int32_t n, int32_t k, const double *A, int64_t lda,
                             const double *B, int64_t ldb, double *C, int64_t ldc, void *dev_buf,
                             size_t dev_bytes, int64_t block, hipStream_t stream) {
    if (m < 0 || n < 0 || k < 0 || block < 0 || block % 128 != 0) return TCU_ERR_ARG;
    if ((m > 0 && n > 0 && C == nullptr) || (m > 0 && k > 0 && A == nullptr) ||
        (k > 0 && n > 0 && B == nullptr))
        return TCU_ERR_ARG;
    if ((m > 0 && lda < k) || (k > 0 && ldb < n) || (m > 0 && ldc < n)) return TCU_ERR_ARG;
    if (m == 0 || n == 0) return TCU_OK;
    const int64_t b = block ? block : ooc_block(dev_bytes);
    if (b == 0 || dev_buf == nullptr || ((uintptr_t)dev_buf % kAlign) != 0 ||
        (size_t)b * (size_t)b * 48 > dev_bytes)
        return TCU_ERR_WORKSPACE;
    return hip_status(
        run_gemm_f64_host(m, n, k, A, lda, B, ldb, C, ldc, dev_buf, dev_bytes, b, stream));
}

tcu_status tcu_sync_status(void *ws, hipStream_t stream, tcu_status_info *info) {
    if (ws == nullptr || ((uintptr_t)ws % kAlign) != 0) return TCU_ERR_WORKSPACE;
    StatusBlock host;
    TCU_TRY(hipMemcpyAsync(&host, ws, sizeof(host), hipMemcpyDeviceToHost, stream));
    TCU_TRY(hipStreamSynchronize(stream));
    if (info != nullptr) {
        info->flags = host.flags;
        info->slices = host.slices;
        info->skipped_a = host.skipped_a;
        info->skipped_b = host.skipped_b;
        info->bits = host.bits;
        info->need = host.need;
        info->exceptions = host.exceptions;
    }
    if (host.flags & kFlagNonFinite) return TCU_ERR_NONFINITE;
    if (host.flags & kFlagKeyRange) return TCU_ERR_KEY_RANGE;
    if (host.flags & kFlagCountRange) return TCU_ERR_COUNT_RANGE;
    return TCU_OK;
}

const char *tcu_status_str(tcu_status s) {
    switch (s) {
        case TCU_OK: return "ok";
        case TCU_ERR_ARG: return "invalid argument";
        case TCU_ERR_KEY_RANGE: return "record with out-of-range key or group (skipped)";
        case TCU_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case TCU_ERR_INFEASIBLE: return "requested tolerance not reachable by the mixed form";
        case TCU_ERR_NONFINITE: return "non-finite value in the mixed form";
        case TCU_ERR_HIP: return "HIP runtime error";
        case TCU_ERR_COUNT_RANGE: return "a pair count exceeded int32 (stored as INT32_MAX)";
    }
    return "unknown status";
}

const char *tcu_version(void) { return "tcudb-mi355x 0.1 (gfx950)"; }

}  // extern "C"
