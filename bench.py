"""Benchmark of the join-aggregate-as-GEMM operator (TCUDB, Section 5.4.1
workload: the matrix multiplication query over dense synthetic tables).

Headline (`value`): the largest workload on one GPU, the paper's largest MM
query: 2^30 records per table (N = 32768), FP32 values drawn from N(0,1)
with 5% of them multiplied by 1e3 (seed 4).  One step = the forward
(encode A -> X, encode B -> Y, certified plan, C = X Y) plus the adjoint
with activation checkpointing (X and Y re-encoded from the records, dX =
W Y^T and dY = X^T W, gathers to the records), in the residue form (int8
residues on the matrix cores, Chinese-remainder reconstruction in FP64)
with the per-cell guarantee |C - C*| <= 1e-12 (|X||Y|).  The FP64 form on
the same step is the comparator.  Inputs are resident in HBM.

The other legs of the same JSON line: the 2^24-record workloads (FP64 on
U[-1,1), seed 2; every mixed form on log-uniform values, seed 3), the
forward at 2^14 and 2^20 records (seeds 0 and 1), the library FP64 GEMM
ceiling (torch.matmul), the library int8 GEMM at the headline size
(torch._int_mm), measured matrix-core rates, and the query family.

The dominant kernel's duration is measured inside the timed steps: the
library records HIP events around every launch of its matrix-core product
kernels on the stream each launch runs on (tcu_trace_launches).

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--legs all]
"""
import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published dense peaks
PEAK_F64_MFMA_TFLOPS = 78.6
PEAK_I8_MFMA_TOPS = 5000.0
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
TOL = 1e-12

METRIC = "elements/sec fwd & fwd+adjoint at 1 GPU; % HBM/MFMA roofline; err vs FP64"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_digest(path):
    """SHA-256 of a C/HIP source with its comments, trailing blanks and empty
    lines removed: it changes when the code does, not when a comment does."""
    import hashlib
    import re
    text = open(path, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [ln.rstrip() for ln in text.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln).encode()).hexdigest()


def counter_traffic(summary, key, source):
    """HBM bytes per launch of one kernel from a committed counter summary
    under profiles/ (a line `traffic: <key>=<bytes> code_sha256=<digest>`,
    FETCH_SIZE + WRITE_SIZE scaled by the plain-copy calibration), or None
    when the summary is missing or was taken with different kernel code."""
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
        src = code_digest(os.path.join(ROOT, "paper_2112_07552_amd", "csrc", source))
    except OSError:
        return None
    m = re.search(rf"traffic: {key}=(\d+) code_sha256=([0-9a-f]{{64}})", text)
    if not m or m.group(2) != src:
        return None
    return int(m.group(1))


class Hip:
    """HIP events through the runtime library torch has loaded."""

    def __init__(self):
        self.rt = C.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.rt.hipEventDestroy.argtypes = [C.c_void_p]

    def event(self):
        ev = C.c_void_p()
        if self.rt.hipEventCreate(C.byref(ev)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return ev.value

    def elapsed_ms(self, a, b):
        ms = C.c_float()
        if self.rt.hipEventElapsedTime(C.byref(ms), C.c_void_p(a), C.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def destroy(self, ev):
        self.rt.hipEventDestroy(C.c_void_p(ev))


class LaunchTrace:
    """Records of the library's matrix-core, encode and gather launches made
    inside a `with` block (tcu_trace_launches), with their durations."""

    def __init__(self, hip, capacity=512):
        from paper_2112_07552_amd import _lib
        self.hip, self.L = hip, _lib.load()
        self.recs = (_lib.tcu_launch_record * capacity)()
        for r in self.recs:
            r.begin, r.end = hip.event(), hip.event()
        self.count = C.c_int32(0)
        self.capacity = capacity

    def __enter__(self):
        from paper_2112_07552_amd import _lib
        _lib.check(self.L.tcu_trace_launches(self.recs, self.capacity, C.byref(self.count)),
                   "tcu_trace_launches")
        return self

    def __exit__(self, *exc):
        self.L.tcu_trace_launches(None, 0, None)
        return False

    def launches(self, kernel):
        """[(ms, ops, m, n, k, planes)] of the recorded launches of one kernel
        (call after the stream has finished the work)."""
        out = []
        for r in self.recs[:min(self.count.value, self.capacity)]:
            if r.kernel == kernel:
                out.append((self.hip.elapsed_ms(r.begin, r.end), r.ops, r.m, r.n, r.k, r.planes))
        return out

    def close(self):
        for r in self.recs:
            self.hip.destroy(r.begin)
            self.hip.destroy(r.end)


def launch_stats(launches, per_unit, unit_name):
    """Average duration and rate over recorded launches: `per_unit` is what
    one unit of `ops` is (e.g. 1 FLOP, 1 byte)."""
    if not launches:
        return None
    ms = sum(x[0] for x in launches)
    ops = sum(x[1] for x in launches)
    shapes = sorted({(x[2], x[3], x[4], x[5]) for x in launches})
    return {"launches": len(launches), "avg_ms": ms / len(launches),
            "avg_ops_per_launch": ops / len(launches),
            f"achieved_{unit_name}": ops / (ms * 1e-3) / per_unit,
            "shapes_m_n_k_planes": [list(s) for s in shapes]}


def time_loop(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms


class Operator:
    """One workload's relations and buffers, and the C-ABI calls of a step
    on the current stream (argument marshalling only)."""

    def __init__(self, A, B, W, M, K, N, stream):
        import torch
        from paper_2112_07552_amd import _lib, ops
        self.L, self.ops, self._lib = _lib.load(), ops, _lib
        self.A, self.B, self.W = A, B, W
        self.M, self.K, self.N = M, K, N
        self.relA = ops.make_relation(A.group, A.key, A.val, unique=True)
        self.relB = ops.make_relation(B.group, B.key, B.val, unique=True)
        dev = A.group.device
        self.C = torch.empty((M, N), dtype=torch.float64, device=dev)
        self.dA = torch.empty(A.n, dtype=torch.float64, device=dev)
        self.dB = torch.empty(B.n, dtype=torch.float64, device=dev)
        self.sp = C.c_void_p(stream.cuda_stream)
        self.ws = None
        self.prec = None

    def use(self, precision, backward=True):
        import torch
        self.ws = None
        torch.cuda.empty_cache()
        nb = self.ops.workspace_bytes(self.relA, self.relB, self.M, self.K, self.N, precision,
                                      backward=backward)
        self.ws = self.ops.alloc_workspace(nb, self.A.group.device)
        self.prec = self.ops.PRECISIONS[precision]
        self.precision = precision
        return nb

    def fwd(self):
        self._lib.check(self.L.tcu_join_agg_fwd(
            C.byref(self.relA), C.byref(self.relB), self.M, self.K, self.N, self.prec, TOL,
            C.c_void_p(self.C.data_ptr()), None, C.c_void_p(self.ws.data_ptr()),
            self.ws.numel(), self.sp), "fwd")

    def bwd(self, saved):
        flags = self._lib.TCU_BWD_SAVED_ENCODINGS if saved else 0
        self._lib.check(self.L.tcu_join_agg_bwd(
            C.byref(self.relA), C.byref(self.relB), self.M, self.K, self.N, self.prec, TOL,
            C.c_void_p(self.W.data_ptr()), C.c_void_p(self.dA.data_ptr()),
            C.c_void_p(self.dB.data_ptr()), flags, C.c_void_p(self.ws.data_ptr()),
            self.ws.numel(), self.sp), "bwd")

    def step(self, saved=False):
        self.fwd()
        self.bwd(saved)

    def status(self):
        st, info = self.ops.sync_status(self.ws)
        if st != 0:
            raise RuntimeError(f"{self.precision}: device status {st}: {info}")
        return info

    def release(self):
        import torch
        self.ws = None
        torch.cuda.empty_cache()


def timed_with_trace(hip, fn, steps, warmup, stream, capacity=512):
    """ms per call of fn over `steps` timed calls after `warmup`, with the
    library's launches inside the timed calls recorded."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    tr = LaunchTrace(hip, capacity)
    with tr:
        ms = time_loop(fn, steps, 0, stream)
    torch.cuda.synchronize()
    return ms, tr


def block_reference(A, B, W, N, R, seed):
    """The oracle on an R x R block of C of the N x N x N workload (rows,
    columns and keys drawn at random), with the value gradients of the A
    records in (rows x keys) and the B records in (keys x columns): 3 R^2 N
    multiply-adds, a fraction R^2 / N^2 of one forward + adjoint step.
    The records are selected on the device (selection, no arithmetic of the
    operator) and copied to the host.  Returns the reference, its scales
    (the same sums of absolute values, untimed) and the oracle's time."""
    import numpy as np
    import torch
    from oracle import oracle as orc

    dev = A.group.device
    rng = np.random.default_rng(seed)
    pick = lambda: np.sort(rng.choice(N, R, replace=False))
    rows, cols, keys = pick(), pick(), pick()

    def lut(sel):
        t = torch.full((N,), -1, dtype=torch.int64, device=dev)
        t[torch.as_tensor(sel, device=dev)] = torch.arange(R, device=dev)
        return t

    lr, lc, lk = lut(rows), lut(cols), lut(keys)
    ga, ka = lr[A.group.long()], lk[A.key.long()]
    hb, kb = lc[B.group.long()], lk[B.key.long()]

    def take(mask, *cols_):
        idx = torch.nonzero(mask).flatten()
        return [c[idx].cpu().numpy() for c in cols_] + [idx.cpu().numpy()]

    f64 = lambda v: v.to(torch.float64)
    # forward block: A records with g in rows, B records with h in cols
    a_g, a_k, a_v, _ = take(ga >= 0, ga, A.key, f64(A.val))
    b_h, b_k, b_v, _ = take(hb >= 0, hb, B.key, f64(B.val))
    # dA: A records in rows x keys against B records with k in keys
    sa_g, sa_k, sa_v, ia = take((ga >= 0) & (ka >= 0), ga, ka, f64(A.val))
    bk_h, bk_k, bk_v, _ = take(kb >= 0, B.group, kb, f64(B.val))
    # dB: B records in keys x cols against A records with k in keys
    sb_h, sb_k, sb_v, ib = take((hb >= 0) & (kb >= 0), hb, kb, f64(B.val))
    ak_g, ak_k, ak_v, _ = take(ka >= 0, A.group, ka, f64(A.val))
    Wr = W[torch.as_tensor(rows, device=dev)].cpu().numpy()
    Wc = W[:, torch.as_tensor(cols, device=dev)].contiguous().cpu().numpy()
    del ga, ka, hb, kb
    torch.cuda.empty_cache()
    i32 = lambda x: x.astype(np.int32)
    Rel = orc.Rel
    fa, fb = Rel(i32(a_g), i32(a_k), a_v), Rel(i32(b_h), i32(b_k), b_v)
    ga_, gb_ = Rel(i32(sa_g), i32(sa_k), sa_v), Rel(i32(bk_h), i32(bk_k), bk_v)
    da_, db_ = Rel(i32(ak_g), i32(ak_k), ak_v), Rel(i32(sb_h), i32(sb_k), sb_v)
    absr = lambda r: Rel(r.group, r.key, np.abs(r.val))
    t0 = time.perf_counter()
    Cb, _, used = orc.join_agg(fa, fb, R, N, R)
    gA = orc.grad(ga_, gb_, R, R, N, Wr, "A")
    gB = orc.grad(da_, db_, N, R, R, Wc, "B")
    t_oracle = time.perf_counter() - t0
    Sb, _, _ = orc.join_agg(absr(fa), absr(fb), R, N, R)
    sA = orc.grad(absr(ga_), absr(gb_), R, R, N, np.abs(Wr), "A")
    sB = orc.grad(absr(da_), absr(db_), N, R, R, np.abs(Wc), "B")
    return {"rows": rows, "cols": cols, "C": Cb, "S": Sb, "ia": ia, "gA": gA, "sA": sA,
            "ib": ib, "gB": gB, "sB": sB, "oracle_s": t_oracle, "threads": int(used),
            "R": R}


def block_errors(ref, Cm, dA, dB):
    import numpy as np
    import torch
    dev = Cm.device
    blk = Cm[torch.as_tensor(ref["rows"], device=dev)][:, torch.as_tensor(ref["cols"], device=dev)]
    e = {"C": float(np.max(np.abs(blk.cpu().numpy() - ref["C"]) / ref["S"]))}
    ga = dA[torch.as_tensor(ref["ia"], device=dev)].cpu().numpy()
    gb = dB[torch.as_tensor(ref["ib"], device=dev)].cpu().numpy()
    e["dA"] = float(np.max(np.abs(ga - ref["gA"]) / ref["sA"]))
    e["dB"] = float(np.max(np.abs(gb - ref["gB"]) / ref["sB"]))
    e["max"] = max(e.values())
    e["cells"], e["records_A"], e["records_B"] = int(ref["C"].size), len(ref["ia"]), len(ref["ib"])
    return e


def crt_tile(n):
    """The residue GEMM's tile for an output n columns wide, as the library
    chooses it (256 x 384 from 16384 columns, else 256 x 256)."""
    return "256x384" if n >= 16384 else "256x256"


def largest_edge(budget):
    """The largest N (a multiple of 256) whose headline step fits in `budget`
    bytes: both tables with FP32 values (12 B per record), W, C, dA and dB
    (8 B each per cell or record), and the residue form's workspace with
    backward as the library sizes it for these relations."""
    from paper_2112_07552_amd import _lib

    L = _lib.load()

    def need(n):
        rel = _lib.tcu_relation(n * n, 1, 1, 1, _lib.TCU_F32, _lib.TCU_REL_UNIQUE_CELLS)
        ws = L.tcu_workspace_bytes(C.byref(rel), C.byref(rel), n, n, n, _lib.TCU_PREC_CRT_I8,
                                   _lib.TCU_WS_BACKWARD)
        return 2 * 12 * n * n + 4 * 8 * n * n + ws

    n = 256
    while need(n + 256) <= budget:
        n += 256
    return n


def library_int8(N, stream, steps=3):
    """The vendor library's int8 GEMM (hipBLASLt through torch._int_mm, int32
    sums, operands N x N and N x N transposed, its faster layout here) on one
    modulus-sized product of the headline: a ceiling for the residue GEMM,
    which runs the same contraction per modulus and also reduces its sums to
    residues.  Never on the path."""
    import torch
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    a = torch.randint(-128, 128, (N, N), dtype=torch.int8, device=dev, generator=g)
    b = torch.randint(-128, 128, (N, N), dtype=torch.int8, device=dev, generator=g)
    bt = b.t()
    ms = time_loop(lambda: torch._int_mm(a, bt), steps, 1, stream)
    del a, b, bt
    torch.cuda.empty_cache()
    return {"call": "torch._int_mm int8 x int8^T -> int32 (hipBLASLt)",
            "m_n_k": [N, N, N], "ms": ms, "tops": 2.0 * N ** 3 / (ms * 1e-3) / 1e12}


def leg_headline(args, stream, hip):
    """2^30 records per table (N = 32768, FP32 mixture values, seed 4): the
    residue form's forward + checkpointed adjoint (the headline), its
    forward alone, the FP64 form's step as the comparator, errors of both on
    the oracle's block, and the oracle's own rate on that block."""
    import torch
    from paper_2112_07552_amd import _lib
    from paper_2112_07552_amd import workloads as wl

    dev = torch.device("cuda:0")
    N = args.n5
    log(f"headline: generating 2 x {N * N} records (N = {N})")
    A, B = wl.mm_query(N, N, N, seed=4, values="mixture", dtype=torch.float32, device=dev)
    W = wl.draw_values("uniform", N * N, 1004, 0, device=dev).reshape(N, N)
    torch.cuda.synchronize()
    out = {"workload": f"MM query, dense {N}x{N} tables ({N * N} records each, random order, "
                       f"unique cells), FP32 values N(0,1) with 5% x1e3 outliers, seed 4; "
                       f"dC = U[-1,1) seed 1004; step = forward + adjoint with "
                       f"checkpointing (X, Y re-encoded)",
           "N": N, "records_per_table": N * N}
    ref = None
    if not args.no_check:
        log(f"headline: oracle on a {args.block} x {args.block} block")
        ref = block_reference(A, B, W, N, args.block, seed=4)
        log(f"headline: oracle block took {ref['oracle_s']:.1f} s on {ref['threads']} threads")
    op = Operator(A, B, W, N, N, N, stream)
    # residue form
    ws_bytes = op.use("crt_i8")
    log(f"headline: residue form, workspace {ws_bytes / 2**30:.1f} GiB")
    ms_step, tr = timed_with_trace(hip, op.step, args.steps, args.warmup, stream)
    info = op.status()
    log(f"headline: residue form step {ms_step:.1f} ms, plan of the last product {info}")
    crt = {"ms_fwd_adjoint_checkpointed": ms_step,
           "fwd_adjoint_elements_per_s": N * N / (ms_step * 1e-3),
           "tol": TOL, "plan_last_product": info}
    gemm = launch_stats(tr.launches(_lib.TCU_KERNEL_GEMM_CRT), 1e12, "tops")
    crt["kernels"] = {
        "gemm_crt": gemm,
        "certify": launch_stats(tr.launches(_lib.TCU_KERNEL_CERTIFY), 1e12, "tops"),
        "encode": launch_stats(tr.launches(_lib.TCU_KERNEL_ENCODE), 1e9, "gbs"),
        "gather": launch_stats(tr.launches(_lib.TCU_KERNEL_GATHER), 1e9, "gbs")}
    tr.close()
    ms_fwd = time_loop(op.fwd, max(2, args.steps // 2), 1, stream)
    crt["ms_fwd"] = ms_fwd
    crt["fwd_elements_per_s"] = N * N / (ms_fwd * 1e-3)
    if ref is not None:
        op.step()
        op.status()
        crt["errors_block"] = block_errors(ref, op.C, op.dA, op.dB)
        log(f"headline: residue form errors {crt['errors_block']}")
    out["crt_i8"] = crt
    if args.no_fp64:
        op.release()
        out["gemm_crt"] = gemm
        return out
    # FP64 comparator
    op.use("fp64")
    ms64 = time_loop(op.step, args.fp64_steps, 1, stream)
    op.status()
    f64 = {"ms_fwd_adjoint_checkpointed": ms64,
           "fwd_adjoint_elements_per_s": N * N / (ms64 * 1e-3),
           "tflops_fwd_adjoint": 6.0 * N ** 3 / (ms64 * 1e-3) / 1e12}
    if ref is not None:
        f64["errors_block"] = block_errors(ref, op.C, op.dA, op.dB)
        log(f"headline: fp64 errors {f64['errors_block']}")
    log(f"headline: fp64 step {ms64:.1f} ms")
    out["fp64"] = f64
    crt["speedup_fwd_adjoint_vs_fp64"] = ms64 / ms_step
    if ref is not None:
        crt["equal_accuracy"] = crt["errors_block"]["max"] <= max(TOL, f64["errors_block"]["max"])
        R = ref["R"]
        out["cpu_baseline"] = {
            "value": R * R / ref["oracle_s"], "unit": "elements/s", "cores": ref["threads"],
            "kind": "oracle",
            "sample": f"the FP64 oracle on a {R} x {R} block of C of this workload plus the "
                      f"value gradients of the {len(ref['ia'])} A records in {R} groups x {R} "
                      f"keys and of the {len(ref['ib'])} B records in {R} keys x {R} groups: "
                      f"3 R^2 N = {3 * R * R * N:.3g} multiply-adds, the fraction R^2/N^2 of "
                      f"one forward + adjoint step, {ref['oracle_s']:.1f} s; elements/s = "
                      f"records per table / extrapolated step time"}
    op.release()
    del op, A, B, W
    torch.cuda.empty_cache()
    out["gemm_crt"] = gemm
    lib = library_int8(N, stream)
    if gemm is not None:
        # the residue GEMM's rate per modulus-sized product, against the library's
        lib["residue_gemm_tops"] = gemm["achieved_tops"]
    log(f"headline: library int8 GEMM {lib['ms']:.2f} ms, {lib['tops']:.0f} TOPS")
    out["library_int8_gemm"] = lib
    return out


def leg_2pow24_fp64(args, stream, hip):
    """2^24 records per table, U[-1,1) FP64 values (seed 2): the FP64 form's
    forward + adjoint with saved encodings and with checkpointing, the
    forward alone, the FP64 GEMM launches inside the timed steps, errors on
    an oracle sample, and the library FP64 GEMM (rocBLAS through
    torch.matmul) on the same shape as the ceiling."""
    import numpy as np
    import torch
    from oracle import sample
    from paper_2112_07552_amd import _lib
    from paper_2112_07552_amd import workloads as wl

    dev = torch.device("cuda:0")
    N = 4096
    A, B = wl.mm_query(N, N, N, seed=2, device=dev)
    W = wl.draw_values("uniform", N * N, 1002, 0, device=dev).reshape(N, N)
    op = Operator(A, B, W, N, N, N, stream)
    op.use("fp64")
    out = {"workload": f"MM query, dense {N}x{N} tables ({N * N} records each), U[-1,1) FP64, "
                       f"seed 2; dC = U[-1,1) seed 1002"}
    ms_step, tr = timed_with_trace(hip, lambda: op.step(saved=True), args.steps, args.warmup,
                                   stream)
    out["ms_fwd_adjoint_saved"] = ms_step
    out["fwd_adjoint_elements_per_s"] = N * N / (ms_step * 1e-3)
    out["tflops_fwd_adjoint"] = 6.0 * N ** 3 / (ms_step * 1e-3) / 1e12
    launches = tr.launches(_lib.TCU_KERNEL_GEMM_F64)
    nn = [x for x in launches if x[2:5] == (N, N, N)]
    out["kernels"] = {"gemm_f64_all": launch_stats(launches, 1e12, "tflops"),
                      "encode": launch_stats(tr.launches(_lib.TCU_KERNEL_ENCODE), 1e9, "gbs"),
                      "gather": launch_stats(tr.launches(_lib.TCU_KERNEL_GATHER), 1e9, "gbs")}
    tr.close()
    ms_ck, tr2 = timed_with_trace(hip, lambda: op.step(saved=False), args.steps, args.warmup,
                                  stream)
    tr2.close()
    out["ms_fwd_adjoint_checkpointed"] = ms_ck
    out["checkpointed_elements_per_s"] = N * N / (ms_ck * 1e-3)
    ms_fwd, trf = timed_with_trace(hip, op.fwd, args.steps, args.warmup, stream)
    out["ms_fwd"] = ms_fwd
    out["fwd_elements_per_s"] = N * N / (ms_fwd * 1e-3)
    out["tflops_fwd"] = 2.0 * N ** 3 / (ms_fwd * 1e-3) / 1e12
    fwd_nn = trf.launches(_lib.TCU_KERNEL_GEMM_F64)
    out["kernels"]["gemm_f64_nn_forward"] = launch_stats(fwd_nn, 1e12, "tflops")
    trf.close()
    op.status()
    if not args.no_check:
        op.step(saved=True)
        ref = sample.reference(*_orc_rels(A, B), N, N, N, W.cpu().numpy(), rows=64, cells=2048,
                               records=1024, seed=2)
        out["errors_sample"] = sample.errors(ref, op.C.cpu().numpy(), op.dA.cpu().numpy(),
                                             op.dB.cpu().numpy())
        log(f"2^24 fp64: errors {out['errors_sample']}")
    op.release()
    # the library FP64 GEMM on the same shape: the ceiling, never on the path
    X = torch.rand((N, N), dtype=torch.float64, device=dev)
    Y = torch.rand((N, N), dtype=torch.float64, device=dev)
    Z = torch.empty((N, N), dtype=torch.float64, device=dev)
    ms_lib = time_loop(lambda: torch.matmul(X, Y, out=Z), args.steps, args.warmup, stream)
    out["library_dgemm"] = {"call": "torch.matmul float64 (rocBLAS / hipBLASLt)",
                            "ms": ms_lib,
                            "tflops": 2.0 * N ** 3 / (ms_lib * 1e-3) / 1e12}
    log(f"2^24 fp64: step {ms_step:.3f} ms, fwd {ms_fwd:.3f} ms, library DGEMM {ms_lib:.3f} ms")
    del X, Y, Z, op, A, B, W
    torch.cuda.empty_cache()
    return out


def _orc_rels(A, B):
    import torch
    from oracle import oracle as orc
    f = lambda R: orc.Rel(R.group.cpu().numpy(), R.key.cpu().numpy(),
                          R.val.cpu().to(torch.float64).numpy())
    return f(A), f(B)


def leg_2pow24_mixed(args, stream, hip):
    """2^24 records per table, values log-uniform in magnitude on [1e-4, 1e4]
    with random sign (seed 3): every form's forward and forward + adjoint
    (saved encodings), its plan, the dominant kernel's launches, and errors
    on the oracle's sample (512 whole rows of C, 4096 cells, Freivalds over
    all of C, 4096 + 4096 gradient records)."""
    import torch
    from oracle import sample
    from paper_2112_07552_amd import _lib
    from paper_2112_07552_amd import workloads as wl

    dev = torch.device("cuda:0")
    N = 4096
    A, B = wl.mm_query(N, N, N, seed=3, values="loguniform", device=dev)
    W = wl.draw_values("uniform", N * N, 1003, 0, device=dev).reshape(N, N)
    out = {"workload": f"MM query, dense {N}x{N} tables ({N * N} records each), values "
                       f"log-uniform on [1e-4, 1e4] with random sign, seed 3; dC = U[-1,1) "
                       f"seed 1003; forward and forward + adjoint (saved encodings)"}
    ref = None
    if not args.no_check:
        t0 = time.perf_counter()
        ref = sample.reference(*_orc_rels(A, B), N, N, N, W.cpu().numpy(), seed=3)
        out["oracle_sample_s"] = time.perf_counter() - t0
        log(f"2^24 mixed: oracle sample {out['oracle_sample_s']:.1f} s")
    op = Operator(A, B, W, N, N, N, stream)
    kernel = {"fp64": (_lib.TCU_KERNEL_GEMM_F64, 1e12, "tflops"),
              "crt_i8": (_lib.TCU_KERNEL_GEMM_CRT, 1e12, "tops"),
              "split_i8": (_lib.TCU_KERNEL_GEMM_SPLIT, 1e12, "tops"),
              "split_bf16": (_lib.TCU_KERNEL_GEMM_SPLIT, 1e12, "tflops")}
    for precision in [f for f in ("fp64", "crt_i8", "split_i8", "split_bf16") if f in args.forms]:
        op.use(precision)
        ms_fwd, trf = timed_with_trace(hip, op.fwd, args.steps, args.warmup, stream)
        trf.close()
        ms_step, tr = timed_with_trace(hip, lambda: op.step(saved=True), args.steps,
                                       args.warmup, stream)
        info = op.status()
        kid, unit, name = kernel[precision]
        e = {"ms_fwd": ms_fwd, "ms_fwd_adjoint": ms_step,
             "fwd_elements_per_s": N * N / (ms_fwd * 1e-3),
             "fwd_adjoint_elements_per_s": N * N / (ms_step * 1e-3),
             "effective_fp64_tflops_fwd": 2.0 * N ** 3 / (ms_fwd * 1e-3) / 1e12,
             "plan_last_product": info,
             "dominant_kernel": launch_stats(tr.launches(kid), unit, name)}
        if precision != "fp64":
            e["certify_kernel"] = launch_stats(tr.launches(_lib.TCU_KERNEL_CERTIFY), 1e12, "tops")
        tr.close()
        if ref is not None:
            op.step(saved=True)
            op.status()
            e["errors_sample"] = sample.errors(ref, op.C.cpu().numpy(), op.dA.cpu().numpy(),
                                               op.dB.cpu().numpy())
        log(f"2^24 mixed {precision}: fwd {ms_fwd:.3f} ms, fwd+adj {ms_step:.3f} ms, "
            f"plan {info}, errors {e.get('errors_sample')}")
        out[precision] = e
    base = out.get("fp64")
    for precision in [f for f in ("crt_i8", "split_i8", "split_bf16") if f in out]:
        if base is None:
            break
        e = out[precision]
        e["speedup_fwd_vs_fp64"] = base["ms_fwd"] / e["ms_fwd"]
        e["speedup_fwd_adjoint_vs_fp64"] = base["ms_fwd_adjoint"] / e["ms_fwd_adjoint"]
        if ref is not None:
            e["equal_accuracy"] = e["errors_sample"]["max"] <= max(
                TOL, base["errors_sample"]["max"])
    op.release()
    del op, A, B, W
    torch.cuda.empty_cache()
    return out


def leg_forward_small(args, stream, hip, N, seed):
    """The FP64 forward at N^2 records per table (U[-1,1), the given seed):
    time, rate, the encode kernel's algorithmic bandwidth, and the error
    against the whole oracle C."""
    import numpy as np
    import torch
    from oracle import oracle as orc
    from paper_2112_07552_amd import _lib
    from paper_2112_07552_amd import workloads as wl

    dev = torch.device("cuda:0")
    A, B = wl.mm_query(N, N, N, seed=seed, device=dev)
    op = Operator(A, B, A.val[:1].reshape(1, 1), N, N, N, stream)
    op.use("fp64", backward=False)
    steps = max(args.steps, 50)
    ms, tr = timed_with_trace(hip, op.fwd, steps, args.warmup, stream, capacity=4 * steps)
    out = {"workload": f"MM query, dense {N}x{N} tables ({N * N} records each), U[-1,1) FP64, "
                       f"seed {seed}; forward",
           "ms_fwd": ms, "fwd_elements_per_s": N * N / (ms * 1e-3),
           "encode": launch_stats(tr.launches(_lib.TCU_KERNEL_ENCODE), 1e9, "gbs"),
           "gemm_f64": launch_stats(tr.launches(_lib.TCU_KERNEL_GEMM_F64), 1e12, "tflops")}
    tr.close()
    op.status()
    # the same forward captured once in a HIP graph and replayed: the launches
    # of its few small kernels no longer go through the runtime one by one
    gs = torch.cuda.Stream(device=dev)
    opg = Operator(A, B, A.val[:1].reshape(1, 1), N, N, N, gs)
    opg.ws, opg.prec, opg.precision = op.ws, op.prec, op.precision
    with torch.cuda.stream(gs):
        opg.fwd()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        opg.fwd()
    with torch.cuda.stream(gs):
        ms_g = time_loop(graph.replay, steps, args.warmup, gs)
    torch.cuda.synchronize()
    op.status()
    out["graph"] = {"ms_fwd": ms_g, "fwd_elements_per_s": N * N / (ms_g * 1e-3)}
    del graph, opg
    if not args.no_check:
        RA, RB = _orc_rels(A, B)
        Co, _, _ = orc.join_agg(RA, RB, N, N, N)
        So, _, _ = orc.join_agg(orc.Rel(RA.group, RA.key, np.abs(RA.val)),
                                orc.Rel(RB.group, RB.key, np.abs(RB.val)), N, N, N)
        out["err_cw_full"] = float(np.max(np.abs(op.C.cpu().numpy() - Co) / So))
    log(f"forward N={N}: {ms:.4f} ms, in a graph {ms_g:.4f} ms, err {out.get('err_cw_full')}")
    op.release()
    return out


PEAK_PROBE_KINDS = {"fp64_tflops": 0, "i8_random_bytes_tops": 1, "i8_constant_bytes_tops": 2}


def measured_peaks(stream, iters=2048, reps=5):
    """Matrix-core rates of register-only loops on this chip (FP64 16x16x4;
    int8 32x32x32 on uniformly random bytes, the residue form's operand
    statistics, and on near-constant bytes), TFLOP/s or TOPS: context for
    the published peaks, which the roofline fractions use."""
    import torch
    from paper_2112_07552_amd import _lib

    L = _lib.load()
    out_buf = torch.empty(L.tcu_mfma_peak_out_bytes(), dtype=torch.uint8, device="cuda:0")
    sp = C.c_void_p(stream.cuda_stream)
    res = {}
    for name, kind in PEAK_PROBE_KINDS.items():
        def probe(kind=kind):
            _lib.check(L.tcu_mfma_peak(kind, iters, C.c_void_p(out_buf.data_ptr()), sp), "peak")
        ms = time_loop(probe, reps, 1, stream)
        res[name] = L.tcu_mfma_peak_ops(kind, iters) / (ms * 1e-3) / 1e12
        log(f"measured peak {name}: {res[name]:.1f}")
    return res


def bench_queries(stream, log, steps, warmup):
    """Q1, Q3 and Q4 of Section 3 end to end from raw int64 ID columns
    (dictionary encoding of the join and group columns, then the operator),
    at the microbenchmark shapes of Section 5.2: n records per table with k
    distinct join values, (n, k) = (32768, 32) and (4096, 4096), plus
    (2^24, 32) for the re-associated forms.  B.Val has 32 distinct values.
    Q1 returns the n x n pair-count matrix; Q3 is timed in the
    re-associated form and as the literal product 1^T (mat(A) mat(B)^T)."""
    import torch
    from paper_2112_07552_amd import ops
    from paper_2112_07552_amd import workloads as wl

    dev = torch.device("cuda:0")
    out = {}
    for n, k in ((32768, 32), (4096, 4096), (1 << 24, 32)):
        ida = wl.id_column(n, k, 70, 1, device=dev)
        idb = wl.id_column(n, k, 70, 2, device=dev)
        bval = wl.id_column(n, 32, 71, 7, device=dev)
        av = wl.draw_values("uniform", n, 70, 3, device=dev)
        bw = wl.draw_values("uniform", n, 70, 4, device=dev)
        tuples = torch.arange(n, dtype=torch.int32, device=dev)
        ones = torch.ones((1, n), dtype=torch.float64, device=dev)
        none = ida[:0]
        _, ka, kb = ops.dict_encode(ida, idb)
        K = int(max(ka.max(), kb.max())) + 1
        r = {}

        def dict_only():
            ops.dict_encode(ida, idb)

        def q3():
            _, a_k, b_k = ops.dict_encode(ida, idb)
            _, g, _ = ops.dict_encode(bval, none)
            ops.join_agg_row(a_k, av, b_k, g, None, K, 32, with_count=True)

        def q4():
            _, a_k, b_k = ops.dict_encode(ida, idb)
            ops.join_agg_row(a_k, av, b_k, tuples[:0].new_zeros(n), bw, K, 1)

        r["ms_dict"] = time_loop(dict_only, steps, warmup, stream)
        r["ms_q3_reassociated"] = time_loop(q3, steps, warmup, stream)
        r["ms_q4_reassociated"] = time_loop(q4, steps, warmup, stream)
        if n <= 32768:
            _, g, _ = ops.dict_encode(bval, none)

            def q1():
                _, a_k, b_k = ops.dict_encode(ida, idb)
                ops.join_agg_fwd(tuples, a_k, None, b_k, tuples, None, n, K, n, unique=True)

            def q3_literal():
                _, a_k, b_k = ops.dict_encode(ida, idb)
                _, gg, _ = ops.dict_encode(bval, none)
                Cf, _, _ = ops.join_agg_fwd(tuples, a_k, av, b_k, gg, None, n, K, 32)
                ops.gemm_f64(ones, Cf)

            r["ms_q1_count_matrix"] = time_loop(q1, max(2, steps // 4), 1, stream)
            r["ms_q3_literal"] = time_loop(q3_literal, steps, warmup, stream)
        r["records_per_s_q3"] = 2 * n / (r["ms_q3_reassociated"] * 1e-3)
        log(f"queries n={n} k={k}: " + ", ".join(f"{a} {b:.3g}" for a, b in r.items()))
        out[f"n{n}_k{k}"] = r
        del ida, idb, bval, av, bw, tuples, ones, ka, kb
        torch.cuda.empty_cache()
    return out


def bench_multiway(stream, log, steps, warmup):
    """The multi-way join of Section 3.2 (query Q2).  The table conversion
    nonzero() over an 8192 x 8192 FP64 matrix with 1% nonzeros, HBM-bound:
    two passes of 8 B per cell read, 8 B per nonzero written (row, column);
    the call reads the count back to the host, as the next join needs it.
    Q2 end to end (dictionaries, first join, conversion, second join) at
    4096 tuples per table with 512 distinct ID1 and ID2 values."""
    import torch
    from paper_2112_07552_amd import ops
    from paper_2112_07552_amd import workloads as wl

    dev = torch.device("cuda:0")
    out = {}
    n = 8192
    u = wl.uniform01(wl.stream_key(82, 0), torch.arange(n * n, device=dev))
    M = torch.where(u < 0.01, u + 0.5, torch.zeros_like(u)).reshape(n, n)
    del u
    r, _, _ = ops.nonzero(M, capacity=1 << 20)
    nnz = r.numel()

    def nz():
        ops.nonzero(M, capacity=nnz)

    ms = time_loop(nz, steps, warmup, stream)
    moved = 2 * 8 * n * n + 8 * nnz
    out["nonzero_8192x8192_1pct"] = {"ms": ms, "nonzero": nnz, "bytes": moved,
                                     "GB_per_s": moved / (ms * 1e-3) / 1e9,
                                     "frac_of_hbm_peak": moved / (ms * 1e-3) / 8e12}
    log(f"multiway: nonzero {n}x{n} 1%: {ms:.3f} ms, {moved / (ms * 1e-3) / 1e9:.0f} GB/s")
    del M
    t = 4096
    a1 = wl.id_column(t, 512, 83, 1, device=dev)
    b1 = wl.id_column(t, 512, 83, 2, device=dev)
    b2 = wl.id_column(t, 512, 83, 3, device=dev)
    c2 = wl.id_column(t, 512, 83, 4, device=dev)
    pa, _, C3 = ops.join3(a1, b1, b2, c2)
    triples = int(C3.count_nonzero())

    def q2():
        ops.join3(a1, b1, b2, c2)

    ms = time_loop(q2, max(2, steps // 4), 1, stream)
    out["q2_4096_tuples_512_ids"] = {"ms": ms, "ab_pairs": int(pa.numel()),
                                     "result_triples": triples}
    log(f"multiway: Q2 4096 tuples: {ms:.3f} ms, {pa.numel()} pairs, {triples} triples")
    return out


def bench_bsr(stream, log, steps, warmup):
    """The block-sparse form (16 x 16 tiles, empty tiles skipped) against
    the dense form on Q1 pair counts with one record per tuple (Section 5.2,
    many distinct join values): (n tuples, k distinct IDs) = (4096, 4096),
    where both run, and (16384, 2^20), where the dense product would take
    2 n^2 K flops (its time is the model 2 n^2 K / (measured dense FP64
    rate)); plus a road-network-like graph (2^16 nodes, 2 edges per node,
    neighbours within +-40) times a 64-column node-feature relation."""
    import torch
    from paper_2112_07552_amd import ops
    from paper_2112_07552_amd import workloads as wl

    dev = torch.device("cuda:0")
    out = {}
    dense_rate = None
    for n, k in ((4096, 4096), (16384, 1 << 20)):
        ida = wl.id_column(n, k, 72, 1, device=dev)
        idb = wl.id_column(n, k, 72, 2, device=dev)
        _, ka, kb = ops.dict_encode(ida, idb)
        K = int(max(ka.max(), kb.max())) + 1
        t = torch.arange(n, dtype=torch.int32, device=dev)
        r = {"K": K}

        def bsr():
            ops.join_agg_bsr(t, ka, None, kb, t, None, n, K, n, unique=True)

        r["ms_bsr"] = time_loop(bsr, steps, warmup, stream)
        flops = 2.0 * n * n * K
        if n * n * K <= 1 << 40:
            def dense():
                ops.join_agg_fwd(t, ka, None, kb, t, None, n, K, n, unique=True)
            r["ms_dense"] = time_loop(dense, max(2, steps // 4), 1, stream)
            dense_rate = flops / (r["ms_dense"] * 1e-3)
        elif dense_rate is not None:
            r["ms_dense_model"] = flops / dense_rate * 1e3
        log(f"bsr q1 n={n} k={k}: " + ", ".join(f"{a} {b:.4g}" for a, b in r.items()))
        out[f"q1_n{n}_k{k}"] = r
        del ida, idb, ka, kb, t
        torch.cuda.empty_cache()
    nodes = 1 << 16
    E = wl.local_edges(2 * nodes, nodes, 40, 73, 1, device=dev)
    F = wl.random_relation(4 * nodes, 64, nodes, 73, 2, device=dev)

    def graph():
        ops.join_agg_bsr(E.group, E.key, E.val, F.key, F.group, F.val, nodes, nodes, 64)

    r = {"ms_bsr": time_loop(graph, steps, warmup, stream),
         "dense_flops": 2.0 * nodes * nodes * 64}
    log(f"bsr graph 2^16 nodes: {r['ms_bsr']:.3f} ms")
    out["graph_65536_nodes"] = r
    # the cost model's choice next to the crossover (Q1, 4096 tuples)
    choice = {}
    for k in (1024, 2048):
        ida = wl.id_column(4096, k, 72, 1, device=dev)
        idb = wl.id_column(4096, k, 72, 2, device=dev)
        _, ka, kb = ops.dict_encode(ida, idb)
        K = int(max(ka.max(), kb.max())) + 1
        t = torch.arange(4096, dtype=torch.int32, device=dev)
        args = (t, ka, None, kb, t, None, 4096, K, 4096)
        c = {"K": K,
             "ms_dense": time_loop(lambda: ops.join_agg_fwd(*args, unique=True), steps, warmup, stream),
             "ms_bsr": time_loop(lambda: ops.join_agg_bsr(*args, unique=True), steps, warmup, stream),
             "picked": "block_sparse" if ops.block_sparse_preferred(*args) else "dense"}
        c["picked_faster"] = (c["picked"] == "block_sparse") == (c["ms_bsr"] < c["ms_dense"])
        log(f"bsr choice q1 n=4096 k={k}: " + ", ".join(f"{a} {b}" for a, b in c.items()))
        choice[f"q1_n4096_k{k}"] = c
    out["cost_model_choice"] = choice
    return out


def bench_ooc(stream, log, N=32768, dev_gb=24):
    """Section 4.2.3: the N x N x N FP64 product with A, B and C in pinned
    host memory, streamed through dev_gb GB of device memory (the paper's
    24 GB card), against the same product with everything resident in HBM.
    One untimed call, then one timed call of each."""
    import torch
    from paper_2112_07552_amd import ops

    dev = torch.device("cuda:0")
    log(f"ooc: generating two {N}x{N} FP64 matrices in pinned host memory")
    Ad = torch.rand((N, N), dtype=torch.float64, device=dev) * 2 - 1
    Bd = torch.rand((N, N), dtype=torch.float64, device=dev) * 2 - 1
    Ah = torch.empty((N, N), dtype=torch.float64, pin_memory=True)
    Bh = torch.empty((N, N), dtype=torch.float64, pin_memory=True)
    Ch = torch.empty((N, N), dtype=torch.float64, pin_memory=True)
    Ah.copy_(Ad)
    Bh.copy_(Bd)
    Cd = torch.empty((N, N), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    flops = 2.0 * N ** 3
    t_dev = time_loop(lambda: ops.gemm_f64(Ad, Bd, out=Cd), 1, 1, stream)
    del Ad, Bd
    torch.cuda.empty_cache()
    dev_bytes = int(dev_gb * 1e9)
    ops.gemm_f64_host(Ah, Bh, out=Ch, dev_bytes=dev_bytes)   # untimed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ops.gemm_f64_host(Ah, Bh, out=Ch, dev_bytes=dev_bytes)
    t_host = (time.perf_counter() - t0) * 1e3
    b = 128
    while (b + 128) ** 2 * 48 <= dev_bytes:
        b += 128
    nb = -(-N // b)
    link = 8.0 * (2 * N * N * nb + N * N)
    sample = float((Ch[:4, :4].to(dev) - Cd[:4, :4]).abs().max())
    log(f"ooc: device-resident {t_dev:.1f} ms, host-resident {t_host:.1f} ms, block {b}, "
        f"{link / 1e9:.0f} GB over the host link")
    return {"N": N, "device_budget_bytes": dev_bytes, "block": b,
            "ms_device_resident": t_dev, "ms_host_resident": t_host,
            "tflops_device_resident": flops / (t_dev * 1e-3) / 1e12,
            "tflops_host_resident": flops / (t_host * 1e-3) / 1e12,
            "host_link_bytes": link, "host_link_gbs": link / (t_host * 1e-3) / 1e9,
            "max_abs_diff_4x4_vs_device": sample}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--legs", default="all",
                    help="comma-separated: headline, fp64_2pow24, mixed_2pow24, small, peaks, "
                         "queries, ooc (not in 'all'), or all")
    ap.add_argument("--n5", type=int, default=32768,
                    help="edge of the headline workload (records per table = n5^2); 0: the "
                         "largest multiple of 256 whose step fits in 0.85 of the free memory")
    ap.add_argument("--block", type=int, default=256,
                    help="edge of the headline's oracle block (its CPU baseline and errors)")
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="timed FP64 comparator steps at the headline workload")
    ap.add_argument("--no-check", action="store_true",
                    help="skip every oracle check (and the CPU baseline)")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 comparator of the headline workload")
    ap.add_argument("--forms", default="fp64,crt_i8,split_i8,split_bf16",
                    help="forms of the 2^24 mixed leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 512 MiB device copy, the reference that scales "
                         "profiler byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the path is built and "
                                   "measured on a single MI355X); --gpus must be 1"}))
        sys.exit(2)
    legs = set(args.legs.split(","))
    if "all" in legs:
        legs |= {"headline", "fp64_2pow24", "mixed_2pow24", "small", "peaks", "queries"}

    import torch
    from paper_2112_07552_amd import _lib

    _lib.load()  # fails loudly without the HIP library
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    hip = Hip()
    res = {}
    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # reads 512 MiB, writes 512 MiB
        torch.cuda.synchronize()
        del src, dst
    if "headline" in legs:
        if args.n5 == 0:
            args.n5 = largest_edge(0.85 * torch.cuda.mem_get_info(dev)[0])
            log(f"headline: largest edge that fits: N = {args.n5}")
        res["headline"] = leg_headline(args, stream, hip)
    if "fp64_2pow24" in legs:
        res["fp64_2pow24"] = leg_2pow24_fp64(args, stream, hip)
    if "mixed_2pow24" in legs:
        res["mixed_2pow24"] = leg_2pow24_mixed(args, stream, hip)
    if "small" in legs:
        res["forward_2pow14"] = leg_forward_small(args, stream, hip, 128, 0)
        res["forward_2pow20"] = leg_forward_small(args, stream, hip, 1024, 1)
    if "peaks" in legs:
        res["measured_peaks"] = measured_peaks(stream)
    if "queries" in legs:
        q = bench_queries(stream, log, args.steps, args.warmup)
        q["block_sparse"] = bench_bsr(stream, log, args.steps, args.warmup)
        q["multiway"] = bench_multiway(stream, log, args.steps, args.warmup)
        res["queries"] = q
    if "ooc" in legs:
        res["out_of_core"] = bench_ooc(stream, log)

    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "data": "synthetic"}
    if "headline" in res and "fp64" in res["headline"]:
        h = res["headline"]
        crt = h["crt_i8"]
        g = h["gemm_crt"]
        N = h["N"]
        out.update({
            "value": crt["fwd_adjoint_elements_per_s"], "unit": "elements/s",
            "ms_per_step": crt["ms_fwd_adjoint_checkpointed"],
            "dtype": "i8",
            "config": {"workload": h["workload"], "records_per_table": h["records_per_table"],
                       "M": N, "K": N, "N": N, "precision": "crt_i8 (int8 residues, int32 "
                       "sums, FP64 reconstruction)", "tol": TOL,
                       "guarantee": "|C - C*| <= tol (|X||Y|) per cell, certified plan"},
            "fwd_elements_per_s": crt["fwd_elements_per_s"],
            "speedup_vs_fp64_form": crt["speedup_fwd_adjoint_vs_fp64"],
            "err_vs_oracle": {k: v.get("errors_block") for k, v in
                              (("crt_i8", crt), ("fp64", h["fp64"]))},
            "roofline": None if g is None else {
                "bound": "mfma", "achieved": g["achieved_tops"], "peak": PEAK_I8_MFMA_TOPS,
                "unit": "TOPS", "frac": g["achieved_tops"] / PEAK_I8_MFMA_TOPS,
                "traffic": counter_traffic("counters_gemm_crt_mm_query_32768.md", "gemm_crt",
                                           "crt.hip"),
                "kernel": f"gemm_crt_kernel ({crt_tile(N)} tiles; the int8 residue "
                          f"products, one launch per modulus, all of the step's launches)",
                "launches": g["launches"], "avg_ms": g["avg_ms"],
                "ops_per_launch": g["avg_ops_per_launch"],
                "library_int8_gemm_tops": h["library_int8_gemm"]["tops"]},
            "cpu_baseline": h.get("cpu_baseline"),
        })
    out["legs"] = res
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
