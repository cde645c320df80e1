"""Benchmark of the density-fitted J/K build on one MI355X.

One step = one Coulomb build J(D) and one exchange build K(C_occ) through the
C-ABI, on the nao=1024 / naux=4096 / nocc=200 workload (B packed, 4096 x
524800, FP64 or FP32), inputs resident in HBM before timing starts.

Prints one JSON line with the step rate, the exchange rate (TFLOP/s, the
`value`), the Coulomb bandwidth, a roofline entry for the dominant kernel
(K GEMM1) and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm_gbs": 8000.0, "f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def k_flops(naux, nao, nocc):
    """GEMM1 (X = B_P C for every P) + lower-triangle SYRK, algorithmic."""
    return 2.0 * naux * nao * nao * nocc, float(naux) * nocc * nao * (nao + 1)


def cpu_baseline(cfg, R, C, D, rows: int):
    """FP64 oracle on the first `rows` auxiliary rows of the same workload."""
    import oracle
    import synth

    B = synth.B_rows(cfg.seed, R, 0, rows)
    t0 = time.perf_counter()
    r = oracle.rho(B, cfg.nao, D)
    J = np.zeros((cfg.nao, cfg.nao))
    oracle.J_acc(B, cfg.nao, r, J)
    tj = time.perf_counter() - t0
    K = np.zeros((cfg.nao, cfg.nao))
    t0 = time.perf_counter()
    oracle.K_C_acc(B, cfg.nao, C, K)
    tk = time.perf_counter() - t0
    g1, sy = k_flops(rows, cfg.nao, cfg.nocc)
    return {
        "value": (g1 + sy) / tk / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"K(C_occ) and J over aux rows 0..{rows - 1} of {cfg.naux} (nao={cfg.nao}, "
                  f"nocc={cfg.nocc}, FP64); K {tk:.2f} s, J {tj:.2f} s",
        "j_gbs": 2 * rows * cfg.npair * 8 / tj / 1e9,
        "seconds": tk + tj,
    }


def counter_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None for every kernel whose source changed since the counters were taken."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return {}
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return {}
    info = json.loads(m.group(1))
    for src, digest in info["sources"].items():
        f = os.path.join(ROOT, "paper_2506_06661_amd", "csrc", src)
        if hashlib.sha256(open(f, "rb").read()).hexdigest()[:16] != digest:
            return {}
    return info["traffic_bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--cpu-rows", type=int, default=1024,
                    help="aux rows in the CPU-oracle sample (0 = skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2506_06661_amd as pkg
    import synth

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if args.copy_calibration:
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return
    cfg = synth.C2
    t0 = time.time()
    R = synth.positions(cfg)
    C = synth.C_occ(cfg.seed, cfg.nao, cfg.nocc)
    D = 2.0 * C @ C.T
    B = synth.B_full(cfg.seed, R, cfg.naux)
    log(f"generated B {B.shape} in {time.time() - t0:.1f} s")
    dt_code = pkg.DFJK_F64 if args.dtype == "f64" else pkg.DFJK_F32
    Bd64 = torch.from_numpy(B).to("cuda")
    del B
    if dt_code == pkg.DFJK_F64:
        Bd = Bd64
    else:
        Bd = torch.empty(Bd64.shape, dtype=torch.float32, device="cuda")
        pkg.dfjk_quantize(Bd64, Bd, dt_code, Bd64.numel())
        del Bd64
    Cd = torch.from_numpy(C).to("cuda")
    Dd = torch.from_numpy(D).to("cuda")
    J = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    h = pkg.Handle(Bd, cfg.nao, dtype=dt_code)
    torch.cuda.synchronize()
    log(f"inputs on device after {time.time() - t0:.1f} s; workspace {h.workspace_bytes() / 1e9:.2f} GB")

    def step():
        pkg.dfjk_build_J(h.h, Dd, J)
        pkg.dfjk_build_K(h.h, Cd, cfg.nocc, None, K)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    pkg.dfjk_profile(h.h, max(args.steps, 1))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    prof = pkg.dfjk_profile_read(h.h)
    log("per-phase event totals (ms, launches):", prof)

    def avg(ph):
        ms, n = prof[ph]
        return ms / max(n, 1)

    g1_flops, sy_flops = k_flops(cfg.naux, cfg.nao, cfg.nocc)
    jbytes = 2.0 * cfg.naux * cfg.npair * Bd.element_size()
    k_ms, j_ms = avg("K"), avg("J")
    g1_ms, sy_ms = avg("K_gemm1"), avg("K_syrk")
    jr_ms, jo_ms = avg("J_rho"), avg("J_out")
    peak = PEAK[args.dtype]
    traffic = counter_traffic(f"c2-{args.dtype}".replace("-", "_"))
    res = {
        "metric": "DF-K TFLOP/s + J HBM GB/s vs FP64 plain; J/K builds to 1e-6 Eh",
        "value": (g1_flops + sy_flops) / k_ms / 1e9,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"DF J/K build: nao={cfg.nao}, naux={cfg.naux}, nocc={cfg.nocc}, packed B "
                        f"{cfg.naux}x{cfg.npair} {args.dtype}, lattice-decay generator; one J(D) + one "
                        f"K(C_occ) build per step",
            "nao": cfg.nao, "naux": cfg.naux, "nocc": cfg.nocc, "B_dtype": args.dtype,
        },
        "j_hbm_gbs": jbytes / j_ms / 1e6,
        "jk_builds_per_s": 1000.0 / (total_ms / args.steps),
        "phase_ms": {"J": j_ms, "J_rho": jr_ms, "J_out": jo_ms, "K": k_ms, "K_gemm1": g1_ms,
                     "K_syrk": sy_ms, "K_finish": avg("K_finish")},
        "roofline": {
            "kernel": "k_gemm1_f64" if args.dtype == "f64" else "k_gemm1_f32",
            "bound": "mfma",
            "achieved": g1_flops / g1_ms / 1e9,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": g1_flops / g1_ms / 1e9 / peak,
            "traffic": traffic.get("k_gemm1_" + args.dtype),
        },
        "kernels": {
            "k_syrk": {"bound": "mfma", "achieved": sy_flops / sy_ms / 1e9, "peak": peak,
                       "unit": "TFLOP/s", "frac": sy_flops / sy_ms / 1e9 / peak,
                       "traffic": traffic.get("k_syrk_" + args.dtype)},
            "j_rho": {"bound": "hbm", "achieved": jbytes / 2 / jr_ms / 1e6, "peak": PEAK["hbm_gbs"],
                      "unit": "GB/s", "frac": jbytes / 2 / jr_ms / 1e6 / PEAK["hbm_gbs"],
                      "traffic": traffic.get("j_rho_" + args.dtype)},
            "j_out": {"bound": "hbm", "achieved": jbytes / 2 / jo_ms / 1e6, "peak": PEAK["hbm_gbs"],
                      "unit": "GB/s", "frac": jbytes / 2 / jo_ms / 1e6 / PEAK["hbm_gbs"],
                      "traffic": traffic.get("j_out_" + args.dtype)},
        },
    }
    h.close()
    del Bd, Cd, Dd
    if args.cpu_rows > 0:
        log(f"timing the CPU oracle on {args.cpu_rows} aux rows ...")
        res["cpu_baseline"] = cpu_baseline(cfg, R, C, D, args.cpu_rows)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
