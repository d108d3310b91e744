#!/usr/bin/env python3
"""Benchmark: n = 16384 tridiagonal eigensolve on one MI355X.

Workload (value): d, e iid Uniform[-1, 1] (seed 0), n = 16384, leaf 32.  One
step = one complete divide-and-conquer solve (leaves, every merge level,
eigenvalues and the full n x n eigenvector matrix) with inputs resident in HBM.
The chosen form (HSS-compressed Uhat for merges with K >= 4096, FP64 MFMA
otherwise) is timed for `value`; the plain FP64-MFMA form is timed beside it.

Also reported on the same JSON line:
  roofline      -- the dominant kernel of the timed workload, measured live with
                   HIP events on the launch stream (library profiling hooks);
  merge_gemm    -- the merge update product on a large-K merge (the rank-one
                   merge of Sec. 2.2 with poles i/N, N = 16384: K = N), TFLOP/s
                   and fraction of the FP64 MFMA peak;
  supplementary -- the Toeplitz-type matrix (diagonal 2, off-diagonal 1) at
                   n = 16383, where no pole deflates at the top merge;
  cpu_baseline  -- the CPU oracle solving the same matrix on the host cores.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0
PHASES = ["leaf", "deflate", "rotate", "secular", "loewner", "uhat_norm", "uhat_write", "rank", "gemm", "copy",
          "sign", "split_slice", "split_gemm", "hss_sample", "hss_compress", "hss_apply", "adj_gemm", "adj_band"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def merge_table(P, work):
    lib = P.load()
    rows = ctypes.c_int64()
    lib.phdc_merge_table.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.phdc_merge_table(ctypes.c_void_p(work.data_ptr()), 0, None, ctypes.byref(rows))
    n = rows.value
    buf = (ctypes.c_int32 * max(n * 10, 1))()
    lib.phdc_merge_table(ctypes.c_void_p(work.data_ptr()), n, buf, ctypes.byref(rows))
    return np.frombuffer(buf, dtype=np.int32)[: n * 10].reshape(n, 10)


def algorithmic(table):
    """Per-phase algorithmic work of one solve from the merge table.

    gemm: 2 [n1 (k1+k2) + n2 (k2+k3)] K flops (Gu's grouped products, Eq. (6));
    copy: deflated columns read and written, 2 * 8 m bytes each;
    uhat_write: 8 K^2 bytes written;
    rotate: each rotation reads and writes two m-long columns, 32 m bytes.
    """
    m, n1, K, k1, k2, k3, nt1, nt2 = (table[:, i].astype(np.float64) for i in range(8))
    n2 = m - n1
    path = table[:, 8]
    plain = path == 0
    return {
        "gemm_flops": float(np.sum((2 * (n1 * (k1 + k2) + n2 * (k2 + k3)) * K)[plain])),
        "copy_bytes": float(np.sum((nt1 + nt2) * m * 16)),
        "uhat_write_bytes": float(np.sum(K * K * 8)),
        "rotate_bytes": float(np.sum(nt2 * m * 32)),
    }


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def profile_phases(P, fn, reps=2):
    import torch
    lib = P.load()
    lib.phdc_profile_enable.argtypes = [ctypes.c_int]
    lib.phdc_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    torch.cuda.synchronize()
    lib.phdc_profile_read((ctypes.c_double * 32)(), (ctypes.c_int64 * 32)(), 32)
    lib.phdc_profile_enable(1)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    lib.phdc_profile_enable(0)
    ms = (ctypes.c_double * 32)()
    cnt = (ctypes.c_int64 * 32)()
    lib.phdc_profile_read(ms, cnt, 32)
    return {PHASES[i]: (ms[i] / reps, cnt[i] // reps) for i in range(len(PHASES)) if cnt[i]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-supp", action="store_true", help="skip the supplementary large-K measurements")
    ap.add_argument("--only", default="", help="profiling aid: run only 'value', 'gemm' or 'supp'")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not an implementation", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_07526_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    n = 16384
    d_np, e_np = W.uniform(n, seed=0)
    d = torch.tensor(d_np, device=dev)
    e = torch.tensor(e_np, device=dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    qbuf = torch.empty((n, n), dtype=torch.float64, device=dev)
    lib = P.load()
    o_hss = P.opts(gemm_mode=P.GEMM_HSS)
    o_plain = P.opts(gemm_mode=P.GEMM_FP64)
    nb = ctypes.c_size_t()
    lib.phdc_stedc_workspace(n, ctypes.byref(o_hss), ctypes.byref(nb))
    work = P.workspace(nb.value, dev)

    def solve(o):
        def f():
            rc = lib.phdc_stedc(n, P._ptr(d), P._ptr(e), P._ptr(lam), P._ptr(qbuf), n, P._ptr(work), work.numel(),
                                ctypes.byref(o), P._stream())
            if rc != 0:
                raise RuntimeError(f"phdc_stedc returned {rc}")
        return f

    result = {}
    if args.only in ("", "value"):
        log(f"[bench] warmup {args.warmup}, timing {args.steps} solves of uniform n={n} (chosen form)")
        t_hss = timed(solve(o_hss), args.steps, args.warmup)
        st = P.status(work)
        if st != 0:
            raise RuntimeError(f"device status {st}")
        table = merge_table(P, work)
        log(f"[bench] chosen form {t_hss * 1e3:.3f} ms/solve; top merge K={table[-1, 2]}")
        t_plain = timed(solve(o_plain), args.steps, 1)
        log(f"[bench] plain FP64 {t_plain * 1e3:.3f} ms/solve")
        # accuracy of the timed solve
        Qd = qbuf.t()
        nrm = float(lam.abs().max())
        orth = float((Qd.T @ Qd - torch.eye(n, dtype=torch.float64, device=dev)).abs().max())
        R = d[:, None] * Qd - Qd * lam[None, :]
        R[:-1] += e[:, None] * Qd[1:]
        R[1:] += e[:, None] * Qd[:-1]
        res = float(torch.linalg.norm(R) / (n * nrm))
        del R
        log(f"[bench] orthogonality {orth:.2e} residual {res:.2e}")
        phases = profile_phases(P, solve(o_plain))
        alg = algorithmic(table)
        log("[bench] phases (ms/solve): " + ", ".join(f"{k}={v[0]:.3f}" for k, v in phases.items()))
        result.update(t_hss=t_hss, t_plain=t_plain, orth=orth, res=res, phases=phases, alg=alg, table=table)

    merge_gemm = None
    if args.only in ("", "gemm") and not args.no_supp:
        N = 16384
        D, z, rho, Q1, Q2 = W.fig3_merge(N, seed=0, with_q=True)
        Dt = torch.tensor(D, device=dev)
        zt = torch.tensor(z, device=dev)
        Q1c, ld1 = P._colmajor(torch.tensor(Q1, device=dev))
        Q2c, ld2 = P._colmajor(torch.tensor(Q2, device=dev))
        del Q1, Q2
        lamm = torch.empty(N, dtype=torch.float64, device=dev)
        qm = torch.empty((N, N), dtype=torch.float64, device=dev)
        lib.phdc_merge_workspace(N // 2, N - N // 2, ctypes.byref(o_plain), ctypes.byref(nb))
        wm = P.workspace(nb.value, dev)

        def mg():
            rc = lib.phdc_merge(N // 2, N - N // 2, P._ptr(Dt), P._ptr(zt), rho, P._ptr(Q1c), ld1, P._ptr(Q2c), ld2,
                                P._ptr(lamm), P._ptr(qm), N, P._ptr(wm), wm.numel(), ctypes.byref(o_plain),
                                P._stream())
            if rc != 0:
                raise RuntimeError(f"phdc_merge returned {rc}")
        log(f"[bench] merge N={N} (poles i/N): warmup")
        mg()
        torch.cuda.synchronize()
        ph = profile_phases(P, mg, reps=2)
        tab = merge_table(P, wm)
        alg = algorithmic(tab)
        gemm_ms = ph["gemm"][0]
        tf = alg["gemm_flops"] / (gemm_ms * 1e-3) / 1e12
        merge_gemm = {"workload": f"rank-one merge, poles i/N, N={N}, K={int(tab[0, 2])}", "tflops": round(tf, 2),
                      "frac_fp64_mfma_peak": round(tf / FP64_PEAK_TFLOPS, 4), "gemm_ms": round(gemm_ms, 3),
                      "merge_ms": round(sum(v[0] for v in ph.values()), 3)}
        log(f"[bench] merge GEMM {tf:.2f} TFLOP/s ({100 * tf / FP64_PEAK_TFLOPS:.1f}% of FP64 MFMA peak)")
        del wm, qm, Q1c, Q2c
        torch.cuda.empty_cache()

    supp = None
    if args.only in ("", "supp") and not args.no_supp:
        ns = 16383
        ds, es = W.toeplitz_121(ns, 1.0)
        dts = torch.tensor(ds, device=dev)
        ets = torch.tensor(es, device=dev)
        lib.phdc_stedc_workspace(ns, ctypes.byref(o_hss), ctypes.byref(nb))
        ws = P.workspace(nb.value, dev)
        ls = torch.empty(ns, dtype=torch.float64, device=dev)
        qs = torch.empty((ns, ns), dtype=torch.float64, device=dev)

        def ss(o):
            def f():
                rc = lib.phdc_stedc(ns, P._ptr(dts), P._ptr(ets), P._ptr(ls), P._ptr(qs), ns, P._ptr(ws),
                                    ws.numel(), ctypes.byref(o), P._stream())
                if rc != 0:
                    raise RuntimeError(f"phdc_stedc returned {rc}")
            return f
        log(f"[bench] Toeplitz-type n={ns}")
        tp = timed(ss(o_plain), 2, 1)
        th = timed(ss(o_hss), 2, 1)
        ph = profile_phases(P, ss(o_plain), reps=1)
        tab = merge_table(P, ws)
        alg = algorithmic(tab)
        tf = alg["gemm_flops"] / (ph["gemm"][0] * 1e-3) / 1e12
        supp = {"workload": f"toeplitz121_n{ns}", "plain_s": round(tp, 5), "chosen_s": round(th, 5),
                "top_K": int(tab[-1, 2]), "gemm_tflops_all_levels": round(tf, 2),
                "gemm_frac_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 4)}
        log(f"[bench] toeplitz plain {tp * 1e3:.1f} ms, chosen {th * 1e3:.1f} ms, GEMM {tf:.1f} TF/s")
        del ws, qs
        torch.cuda.empty_cache()

    if args.only not in ("", "value"):
        return

    # roofline of the dominant kernel class of the timed workload
    phases, alg = result["phases"], result["alg"]
    dom = max(phases.items(), key=lambda kv: kv[1][0])[0]
    ms_dom, cnt_dom = phases[dom]
    if dom == "gemm":
        roof = {"bound": "mfma", "achieved": alg["gemm_flops"] / (ms_dom * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        key = {"copy": "copy_bytes", "uhat_write": "uhat_write_bytes", "rotate": "rotate_bytes"}.get(dom)
        byts = alg.get(key, 0.0) if key else 0.0
        roof = {"bound": "hbm", "achieved": byts / (ms_dom * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["achieved"] = round(roof["achieved"], 3)
    roof["frac"] = round(roof["achieved"] / roof["peak"], 5)
    roof["traffic"] = None
    roof["kernel"] = dom
    roof["launches_per_step"] = int(cnt_dom)
    roof["ms_per_step"] = round(ms_dom, 4)

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"[bench] CPU oracle: one full solve of the same matrix on {threads} threads")
        orc = oracle.get()
        t0 = time.perf_counter()
        lref, _, _ = orc.stedc(d_np, e_np)
        tc = time.perf_counter() - t0
        err = float(np.abs(lam.cpu().numpy() - lref).max())
        cpu = {"value": round(tc, 3), "unit": "s", "cores": threads, "kind": "oracle",
               "sample": f"one full solve, uniform n={n} (whole workload)", "max_abs_dlambda_vs_gpu": err}
        log(f"[bench] oracle {tc:.2f} s; max |lambda_gpu - lambda_oracle| = {err:.2e}")

    t_val = result["t_hss"]
    line = {
        "metric": "n=16384 eigensolve time (s) + merge-GEMM % MFMA peak, plain vs chosen form",
        "value": round(t_val, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_val * 1e3, 4),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uniform_n16384", "n": n, "dist": "d,e iid U[-1,1] seed 0", "leaf": 32,
                   "chosen_form": "hss (K>=4096) else fp64-mfma", "top_merge_K": int(result["table"][-1, 2])},
        "plain_fp64_s": round(result["t_plain"], 6),
        "accuracy": {"orth_max": result["orth"], "residual": result["res"]},
        "phases_ms": {k: round(v[0], 4) for k, v in phases.items()},
        "roofline": roof,
        "merge_gemm": merge_gemm,
        "supplementary": supp,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
