"""Run one contraction kernel of the library alone, a few times, for profiler
counter passes (rocprofv3 --pmc ... -- python3 -m paper_2112_07552_amd.kernel_driver W N R).

W: nn, nt, tn or tt runs tcu_gemm_f64 on N x N operands (uniform [-1, 1));
   fp64, split_i8, split_bf16 or crt_i8 runs the forward operator on the MM-query
   tables of N x N records with log-uniform values (seed 3), tol 1e-12.
N: matrix edge (default 4096).  R: repetitions (default 3).
A fifth argument "calib" adds one plain 512 MiB device copy (runtime copy
kernels), whose counter readings calibrate the memory counters of the pass.
"""
import ctypes as C
import sys

import torch

from . import _lib, ops
from . import workloads as wl


def main(argv):
    which = argv[1]
    N = int(argv[2]) if len(argv) > 2 else 4096
    reps = int(argv[3]) if len(argv) > 3 else 3
    dev = torch.device("cuda:0")
    L = _lib.load()
    sp = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    if which in ("nn", "nt", "tn", "tt"):
        X = wl.draw_values("uniform", N * N, 5, 1, device=dev).reshape(N, N)
        Y = wl.draw_values("uniform", N * N, 5, 2, device=dev).reshape(N, N)
        G = torch.empty((N, N), dtype=torch.float64, device=dev)
        ta, tb = {"nn": (0, 0), "nt": (0, 1), "tn": (1, 0), "tt": (1, 1)}[which]
        for _ in range(reps):
            _lib.check(L.tcu_gemm_f64(ta, tb, N, N, N, C.c_void_p(X.data_ptr()), N,
                                      C.c_void_p(Y.data_ptr()), N, C.c_void_p(G.data_ptr()), N,
                                      sp), "tcu_gemm_f64")
    else:
        A, B = wl.mm_query(N, N, N, seed=3, values="loguniform", device=dev)
        for _ in range(reps):
            ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, N, N, N,
                             precision=which, tol=1e-12, unique=True)
    if len(argv) > 4 and argv[4] == "calib":
        src = torch.empty(64 << 20, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)  # reads 512 MiB, writes 512 MiB
    torch.cuda.synchronize()
    print("done", which, N, reps, flush=True)


if __name__ == "__main__":
    main(sys.argv)
