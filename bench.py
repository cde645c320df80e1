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


def host_info():
    """CPU model (lscpu, else /proc/cpuinfo) and the cores this process may use."""
    import subprocess

    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if not model:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}


def _oracle_jk(oracle, B, nao, C, D):
    """(seconds for J, seconds for K) of one oracle J(D) + K(C) over the rows of B."""
    t0 = time.perf_counter()
    r = oracle.rho(B, nao, D)
    J = np.zeros((nao, nao))
    oracle.J_acc(B, nao, r, J)
    tj = time.perf_counter() - t0
    K = np.zeros((nao, nao))
    t0 = time.perf_counter()
    oracle.K_C_acc(B, nao, C, K)
    return tj, time.perf_counter() - t0


def cpu_baseline(cfg, R, C, D, rows: int, rows_1t: int = 32):
    """FP64 oracle on the host: the first `rows` auxiliary rows of the same
    workload with all threads (median of 3), the first `rows_1t` rows with one
    thread, and the nao=64 workload in full with one thread and with all
    (median of 3 each)."""
    import oracle
    import synth

    threads = oracle.num_threads()
    B = synth.B_rows(cfg.seed, R, 0, rows)
    runs = [_oracle_jk(oracle, B, cfg.nao, C, D) for _ in range(3)]
    tj = float(np.median([r[0] for r in runs]))
    tk = float(np.median([r[1] for r in runs]))
    g1, sy = k_flops(rows, cfg.nao, cfg.nocc)
    oracle.set_num_threads(1)
    try:
        tj1, tk1 = _oracle_jk(oracle, B[:rows_1t], cfg.nao, C, D)
        c1 = synth.C1
        R1 = synth.positions(c1)
        B1 = synth.B_full(c1.seed, R1, c1.naux)
        C1 = synth.C_occ(c1.seed, c1.nao, c1.nocc)
        D1 = 2.0 * C1 @ C1.T
        c1_1t = float(np.median([sum(_oracle_jk(oracle, B1, c1.nao, C1, D1)) for _ in range(3)]))
    finally:
        oracle.set_num_threads(threads)
    c1_all = float(np.median([sum(_oracle_jk(oracle, B1, c1.nao, C1, D1)) for _ in range(3)]))
    g1_1t, sy_1t = k_flops(rows_1t, cfg.nao, cfg.nocc)
    return {
        "value": (g1 + sy) / tk / 1e12,
        "unit": "TFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"K(C_occ) and J over aux rows 0..{rows - 1} of {cfg.naux} (nao={cfg.nao}, "
                  f"nocc={cfg.nocc}, FP64), median of 3: K {tk:.2f} s, J {tj:.2f} s",
        "j_gbs": 2 * rows * cfg.npair * 8 / tj / 1e9,
        "seconds": 3 * (tk + tj),
        **host_info(),
        "one_thread": {
            "k_tflops": (g1_1t + sy_1t) / tk1 / 1e12, "j_gbs": 2 * rows_1t * cfg.npair * 8 / tj1 / 1e9,
            "sample": f"aux rows 0..{rows_1t - 1}, one run: K {tk1:.2f} s, J {tj1:.2f} s"},
        "nao64_jk_seconds": {"one_thread_median_of_3": c1_1t, "all_threads_median_of_3": c1_all,
                             "workload": f"nao={synth.C1.nao}, naux={synth.C1.naux}, "
                                         f"nocc={synth.C1.nocc}, one J + one K"},
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


TRAFFIC_SOURCES = ("k_kernels.hip", "j_kernels.hip", "mma.h")


def traffic_summary(fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str,
                    first: int, command: str) -> str:
    """Markdown summary of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE
    in KiB per dispatch) of the default nao=1024 FP64 workload, scaled by
    what the same counters read for a 1 GiB device copy (--copy-calibration).
    Per kernel: the mean over its first `first` dispatches (the warm-up and
    timed steps; later dispatches of the same kernel belong to the extra
    measurements).  The JSON block is what counter_traffic reads."""
    import collections
    import csv
    import hashlib
    import re

    def per_dispatch(d, counter):
        path = os.path.join(d, "run_counter_collection.csv")
        vals = collections.OrderedDict()
        names = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            k = int(r["Dispatch_Id"])
            vals[k] = vals.get(k, 0.0) + float(r["Counter_Value"])
            m = re.search(r"(\w+)(<[^()]*>)?\(", r["Kernel_Name"])
            names[k] = (m.group(1) + (m.group(2) or "")) if m else r["Kernel_Name"][:60]
        out = collections.OrderedDict()
        for k in sorted(vals):
            out.setdefault(names[k], []).append(vals[k])
            first_id.setdefault(names[k], k)
        return out

    first_id = {}  # kernel name -> its first dispatch id (FETCH_SIZE run)

    gib = float(1 << 30)
    cf = per_dispatch(copy_fetch_dir, "FETCH_SIZE")
    cw = per_dispatch(copy_write_dir, "WRITE_SIZE")
    ck = [k for k in cf if "copyBuffer" in k][0]
    f_scale = gib / (float(np.median(cf[ck])) * 1024.0)
    w_scale = gib / (float(np.median(cw[ck])) * 1024.0)
    wr = per_dispatch(write_dir, "WRITE_SIZE")
    first_id.clear()
    fe = per_dispatch(fetch_dir, "FETCH_SIZE")
    k_fin_first = first_id.get("k_syrk_finish<double>", 1 << 62)
    cfg = __import__("synth").C2
    npair = cfg.nao * (cfg.nao + 1) // 2
    b_bytes = cfg.naux * npair * 8.0
    x_bytes = cfg.naux * cfg.nocc * cfg.nao * 8.0
    mins = {"j_rho_f64": b_bytes, "j_out_f64": b_bytes, "k_syrk_f64": x_bytes}
    rows, traffic = [], {}
    g1_total = 0.0
    for name, fv in fe.items():
        if name not in wr or name.startswith(("at::", "void at::")) or "rocclr" in name:
            continue
        f_kib = float(np.mean(fv[:first]))
        w_kib = float(np.mean(wr[name][:first]))
        byts = f_kib * 1024.0 * f_scale + w_kib * 1024.0 * w_scale
        key = None
        if name.startswith("k_gemm1<double") and first_id[name] < k_fin_first:
            # the launches of the J/K step's K (the first K finish follows them)
            g1_total += byts
            key = "k_gemm1_f64 launch " + name
        elif name.startswith("j_rho_f64<"):
            key = "j_rho_f64"
        elif name.startswith("j_out_f64<") and name.endswith("false>"):
            key = "j_out_f64"
        elif name.startswith("k_syrk<double, 0"):
            key = "k_syrk_f64"
        mn = mins.get(key)
        rows.append(f"| `{name}` | {f_kib:.4g} | {w_kib:.4g} | {byts:.4g} | "
                    f"{'%.4g' % mn if mn else ''} | {'%.3f' % (byts / mn) if mn else ''} |")
        traffic[key or name] = byts
    traffic["k_gemm1_f64"] = g1_total
    g1_min = b_bytes + x_bytes
    digests = {src: hashlib.sha256(open(os.path.join(ROOT, "paper_2506_06661_amd", "csrc", src), "rb").read())
               .hexdigest()[:16] for src in TRAFFIC_SOURCES}
    info = {"workload": "c2-f64", "sources": digests, "traffic_bytes": traffic}
    lines = [
        f"# HBM traffic per launch: DF J/K build, nao={cfg.nao} naux={cfg.naux} nocc={cfg.nocc}, FP64 B (MI355X)",
        "",
        "Commands (from the repository root; one counter per run), then this summary:",
        "",
        "```", command, "```", "",
        f"Calibration: a 1 GiB device copy (`{ck}`) reads FETCH_SIZE = {np.median(cf[ck]):.0f} KiB and "
        f"WRITE_SIZE = {np.median(cw[ck]):.0f} KiB,",
        f"so FETCH_SIZE is scaled by {f_scale:.3f} and WRITE_SIZE by {w_scale:.3f} to give bytes. Values are "
        f"the mean over each kernel's first {first} dispatches (warm-up and timed steps).",
        "",
        "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled HBM bytes | minimum algorithmic bytes | ratio |",
        "|---|---|---|---|---|---|",
        *rows,
        "",
        "Minimum algorithmic bytes: each J pass reads B once (naux*npair*8); the GEMM1 phase reads B once and "
        "writes X (naux*nocc*nao*8); the SYRK reads X once.",
        f"GEMM1 phase (all launches of a step): {g1_total:.4g} bytes against a minimum of {g1_min:.4g} "
        f"({g1_total / g1_min:.2f}x): each launch reads every packed element for both triangles it serves.",
        "",
        "Machine-readable (read by bench.py while the kernel sources are unchanged):",
        "",
        "```json", json.dumps(info), "```", "",
    ]
    return "\n".join(lines)


def time_steps(pkg, h, Dd, Cd, cfg, steps, warmup):
    """Per-phase event averages over `steps` J+K steps on handle h."""
    import torch

    J = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    for _ in range(warmup):
        pkg.dfjk_build_J(h.h, Dd, J)
        pkg.dfjk_build_K(h.h, Cd, cfg.nocc, None, K)
    torch.cuda.synchronize()
    pkg.dfjk_profile(h.h, max(steps, 1))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    e0.record()
    for a, b, c in ev:
        a.record()
        pkg.dfjk_build_J(h.h, Dd, J)
        b.record()
        pkg.dfjk_build_K(h.h, Cd, cfg.nocc, None, K)
        c.record()
    e1.record()
    torch.cuda.synchronize()
    prof = pkg.dfjk_profile_read(h.h)
    pkg.dfjk_profile(h.h, 0)
    return {"ms_per_step": e0.elapsed_time(e1) / steps,
            "median_ms": {"step": float(np.median([a.elapsed_time(c) for a, b, c in ev])),
                          "J": float(np.median([a.elapsed_time(b) for a, b, c in ev])),
                          "K": float(np.median([b.elapsed_time(c) for a, b, c in ev]))},
            "phase_ms": {k: v[0] / max(v[1], 1) for k, v in prof.items()}}


class C3CpuLeg:
    """CPU-baseline leg of the nao=2048 workload: the FP64 oracle streams the
    same row blocks as the device copy is made (rho and J over every auxiliary
    row, timed), then builds the whole K of the first `slice_rows` rows in FP64
    and on those rows rounded to each stored format (timed).  Each GPU result
    is stated against it: (i) the oracle on the FP64 B, (ii) the oracle on the
    rounded B."""

    def __init__(self, cfg, C, D, slice_rows: int = 64):
        import oracle

        self.o, self.cfg, self.C, self.D, self.ns = oracle, cfg, C, D, slice_rows
        self.rho = np.empty(cfg.naux)
        self.J = np.zeros((cfg.nao, cfg.nao))
        self.t_j = 0.0
        self.slice_B = None

    def feed(self, P0: int, blk: np.ndarray) -> None:
        t0 = time.perf_counter()
        r = self.o.rho(blk, self.cfg.nao, self.D)
        self.o.J_acc(blk, self.cfg.nao, r, self.J)
        self.t_j += time.perf_counter() - t0
        self.rho[P0:P0 + blk.shape[0]] = r
        if P0 == 0:
            self.slice_B = np.ascontiguousarray(blk[:self.ns])

    def slice_refs(self, name: str):
        """Oracle J, rho and K of the slice system: FP64 rows (i) and rows
        rounded to `name` (ii); for the 16-bit exchange option also with C
        rounded to `name` (ii')."""
        o, nao, C, D = self.o, self.cfg.nao, self.C, self.D
        q = {"bf16": o.quantize_bf16, "f16": o.quantize_f16}[name]
        out = {}
        t0 = time.perf_counter()
        for key, Bs, Cs in [("i", self.slice_B, C), ("ii", q(self.slice_B), C), ("ii_k16", None, q(C))]:
            Bs = out["ii"][3] if Bs is None else Bs
            Jr, rr = o.J(Bs, nao, D, return_rho=True)
            out[key] = (Jr, rr, o.K_C(Bs, nao, Cs), Bs)
        self.t_k = time.perf_counter() - t0
        return out

    def report(self, name: str, gpu: dict) -> dict:
        """Errors of the GPU results `gpu` (J, rho over all rows; J, rho, K,
        K16 of the slice) against the oracle."""
        def frob(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))

        def e2(rho_, K_):
            return 0.5 * float(rho_ @ rho_) - 0.25 * float(np.sum(self.D * K_))

        ref = self.slice_refs(name)
        J, rho = gpu["J"], gpu["rho"]
        ej, ej_o = 0.5 * float(rho @ rho), 0.5 * float(self.rho @ self.rho)
        res = {"J_frob_i": frob(J, self.J), "J_maxrel_i": float(np.abs(J - self.J).max() / np.abs(self.J).max()),
               "E_J_Eh": ej_o, "E_J_err_i_Eh": ej - ej_o}
        sl = {"aux_rows": self.ns}
        for key in ("i", "ii"):
            Jr, rr, Kr, _ = ref[key]
            sl[f"J_frob_{key}"] = frob(gpu["J_s"], Jr)
            sl[f"K_frob_{key}"] = frob(gpu["K_s"], Kr)
            sl[f"E_2e_err_{key}_Eh"] = e2(gpu["rho_s"], gpu["K_s"]) - e2(rr, Kr)
        sl["E_2e_Eh"] = e2(ref["i"][1], ref["i"][2])
        sl["k16"] = {"K_frob_i": frob(gpu["K16_s"], ref["i"][2]),
                     "K_frob_ii_C_rounded": frob(gpu["K16_s"], ref["ii_k16"][2]),
                     "E_2e_err_i_Eh": e2(gpu["rho_s"], gpu["K16_s"]) - e2(ref["i"][1], ref["i"][2]),
                     "E_2e_err_ii_Eh": e2(gpu["rho_s"], gpu["K16_s"]) - e2(ref["ii_k16"][1], ref["ii_k16"][2])}
        res["slice"] = sl
        return res


def bench_c3(args):
    """nao=2048, naux=8192, nocc=400: B stored in BF16 and in FP16 (34 GB each),
    generated in FP64 row blocks on the host and rounded on the device."""
    import torch

    import paper_2506_06661_amd as pkg
    import synth

    cfg = synth.C3
    R = synth.positions(cfg)
    C = synth.C_occ(cfg.seed, cfg.nao, cfg.nocc)
    D = 2.0 * C @ C.T
    Cd, Dd = torch.from_numpy(C).cuda(), torch.from_numpy(D).cuda()
    out = {}
    g1_flops, sy_flops = k_flops(cfg.naux, cfg.nao, cfg.nocc)
    bufs = {}
    for name, code, tdt in [("bf16", pkg.DFJK_BF16, torch.bfloat16), ("f16", pkg.DFJK_F16, torch.float16)]:
        bufs[name] = (code, torch.empty((cfg.naux, cfg.npair), dtype=tdt, device="cuda"))
    cpu = C3CpuLeg(cfg, C, D) if args.cpu_rows > 0 else None
    t0 = time.time()
    rows = 512
    for P0 in range(0, cfg.naux, rows):
        host_blk = synth.B_rows(cfg.seed, R, P0, rows)
        blk = torch.from_numpy(host_blk).cuda()
        for name, (code, buf) in bufs.items():
            pkg.dfjk_quantize(blk, buf[P0:P0 + rows], code, blk.numel())
        if cpu is not None:
            cpu.feed(P0, host_blk)
        torch.cuda.synchronize()
        log(f"  rows {P0 + rows}/{cfg.naux} after {time.time() - t0:.0f} s")
    del blk, host_blk
    gpu_out = {}
    for name, (code, buf) in bufs.items():
        h = pkg.Handle(buf, cfg.nao, dtype=code)
        r = time_steps(pkg, h, Dd, Cd, cfg, args.steps, args.warmup)
        ph = r["phase_ms"]
        jb = 2.0 * cfg.naux * cfg.npair * 2
        out[name] = {"k_tflops": (g1_flops + sy_flops) / ph["K"] / 1e9, "j_hbm_gbs": jb / ph["J"] / 1e6,
                     "ms_per_step": r["ms_per_step"], "phase_ms": ph,
                     "k_gemm1_frac_of_f32_peak": g1_flops / ph["K_gemm1"] / 1e9 / PEAK["f32"],
                     "j_frac_of_hbm": jb / ph["J"] / 1e6 / PEAK["hbm_gbs"]}
        if cpu is not None:  # results whose errors the CPU leg states
            Jt = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
            rt = torch.empty(cfg.naux, dtype=torch.float64, device="cuda")
            pkg.dfjk_build_J(h.h, Dd, Jt, rt)
            g = {"J": Jt.cpu().numpy(), "rho": rt.cpu().numpy()}
            ns = cpu.ns
            for key, k16 in (("", 0), ("16", 1)):
                o = pkg.dfjk.default_options()
                o.k16 = k16
                hs = pkg.Handle(buf[:ns], cfg.nao, dtype=code, opts=o)
                rs = torch.empty(ns, dtype=torch.float64, device="cuda")
                pkg.dfjk_build_J(hs.h, Dd, Jt, rs)
                g["J_s"], g["rho_s"] = Jt.cpu().numpy(), rs.cpu().numpy()
                pkg.dfjk_build_K(hs.h, Cd, cfg.nocc, None, Jt)
                g[f"K{key}_s"] = Jt.cpu().numpy()
                hs.close()
            gpu_out[name] = g
            del Jt, rt
        h.close()
        # the same build with K on the 16-bit matrix cores (dense 16-bit copy of B)
        opts = pkg.dfjk.default_options()
        opts.k16 = 1
        h16 = pkg.Handle(buf, cfg.nao, dtype=code, opts=opts)
        Kt = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        tc = time.perf_counter()
        pkg.dfjk_build_K(h16.h, Cd, cfg.nocc, None, Kt)  # makes the dense copy
        torch.cuda.synchronize()
        first_ms = (time.perf_counter() - tc) * 1e3
        r16 = time_steps(pkg, h16, Dd, Cd, cfg, args.steps, args.warmup)
        p16 = r16["phase_ms"]
        peak16 = PEAK[name]
        out[name]["k16"] = {"k_tflops": (g1_flops + sy_flops) / p16["K"] / 1e9, "ms_per_step": r16["ms_per_step"],
                            "phase_ms": p16, "first_call_ms_incl_dense_copy": first_ms,
                            "dense_copy_gb": h16.workspace_bytes() / 1e9,
                            "k_gemm1_frac_of_16bit_peak": g1_flops / p16["K_gemm1"] / 1e9 / peak16,
                            "k_syrk_frac_of_16bit_peak": sy_flops / p16["K_syrk"] / 1e9 / peak16}
        h16.close()
        del Kt
        log(name, out[name])
    res = {"metric": "DF-K TFLOP/s + J HBM GB/s vs FP64 plain; J/K builds to 1e-6 Eh",
           "value": out["bf16"]["k_tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": out["bf16"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 (B stored bf16/f16)", "data": "synthetic",
           "config": {"workload": f"DF J/K build: nao={cfg.nao}, naux={cfg.naux}, nocc={cfg.nocc}, packed B "
                                  f"stored BF16 and FP16 (34 GB each), J FP64 accumulation, K on FP32 "
                                  f"matrix cores (k16: on 16-bit matrix cores)", "nao": cfg.nao,
                      "naux": cfg.naux, "nocc": cfg.nocc},
           "bf16": out["bf16"], "f16": out["f16"]}
    if cpu is not None:
        for name in ("bf16", "f16"):
            res[name]["errors_vs_fp64_oracle"] = cpu.report(name, gpu_out[name])
        res["cpu_baseline"] = {
            "value": 2.0 * cfg.naux * cfg.npair * 8 / cpu.t_j / 1e9, "unit": "GB/s (J, FP64 B)",
            "cores": cpu.o.num_threads(), "kind": "oracle", **host_info(),
            "sample": f"rho and J over all {cfg.naux} aux rows in FP64 ({cpu.t_j:.1f} s, streamed in "
                      f"512-row blocks); K of the first {cpu.ns} rows three times (FP64, rounded B, "
                      f"rounded B and C) in {cpu.t_k:.1f} s",
            "k_tflops": 3 * sum(k_flops(cpu.ns, cfg.nao, cfg.nocc)) / cpu.t_k / 1e12}
        res["errors_note"] = ("(i) against the FP64 oracle on the FP64 B, (ii) against the FP64 oracle on the "
                              "rounded B; J and E_J over all rows, the rest on the system of the first "
                              f"{cpu.ns} auxiliary rows (whole J, K and E_2e = E_J + E_K)")
    print(json.dumps(res), flush=True)


def bench_c4(args):
    """256 molecules, nao ~ U{40..400}, naux = 4 nao, nocc = nao // 5, one
    batched build per step (FP32 and BF16 storage); against a loop of
    single-molecule builds and against the untuned tiles."""
    import torch

    import paper_2506_06661_amd as pkg
    import synth

    sizes = synth.batch_sizes()
    res_d = {}
    mols = {}
    t0 = time.time()
    for name, code, tdt in [("f32", pkg.DFJK_F32, torch.float32), ("bf16", pkg.DFJK_BF16, torch.bfloat16)]:
        mols[name] = []
    for i, nao in enumerate(sizes):
        nao = int(nao)
        seed = 4000 + i
        R = synth.cluster_positions(seed, nao)
        B = torch.from_numpy(synth.B_full(seed, R, 4 * nao)).cuda()
        C = synth.C_occ(seed, nao, max(nao // 5, 1))
        Cd = torch.from_numpy(C).cuda()
        Dd = 2.0 * Cd @ Cd.T
        for name, code, tdt in [("f32", pkg.DFJK_F32, torch.float32), ("bf16", pkg.DFJK_BF16, torch.bfloat16)]:
            Bq = torch.empty(B.shape, dtype=tdt, device="cuda")
            pkg.dfjk_quantize(B, Bq, code, B.numel())
            mols[name].append({"B": Bq, "nao": nao, "D": Dd, "C": Cd,
                               "J": torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
                               "K": torch.empty((nao, nao), dtype=torch.float64, device="cuda")})
        del B
    torch.cuda.synchronize()
    log(f"generated {len(sizes)} molecules in {time.time() - t0:.0f} s")
    jbytes = {n: 0.0 for n in mols}
    kfl = 0.0
    for i, nao in enumerate(sizes):
        nao = int(nao)
        npair = nao * (nao + 1) // 2
        g1, sy = k_flops(4 * nao, nao, max(nao // 5, 1))
        kfl += g1 + sy
        jbytes["f32"] += 2 * 4 * nao * npair * 4
        jbytes["bf16"] += 2 * 4 * nao * npair * 2

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for name, code, _ in [("f32", pkg.DFJK_F32, None), ("bf16", pkg.DFJK_BF16, None)]:
        bt = pkg.Batch(mols[name], code)
        untuned = timed(bt.build, args.steps)
        bt.autotune(reps=3, cache_path=None)
        tiles = [bt.tile(b) for b in range(8)]
        eager = timed(bt.build, args.steps)
        bt.capture()
        graph = timed(bt.launch, args.steps)
        k16 = None
        if code != pkg.DFJK_F32:
            # the exchange on the 16-bit matrix cores (GEMM1 on the packed triangle)
            bt.set_k16(True)
            e16 = timed(bt.build, args.steps)
            bt.capture()
            g16 = timed(bt.launch, args.steps)
            k16 = {"graph_ms": g16, "eager_ms": e16, "molecules_per_s": len(sizes) / g16 * 1e3,
                   "k_tflops_aggregate": kfl / g16 / 1e9, "speedup_vs_fp32_exchange": graph / g16,
                   "workspace_gb": bt.workspace_bytes() / 1e9}
        singles = [pkg.Handle(m["B"], m["nao"], dtype=code) for m in mols[name]]

        def loop():
            for hs, m in zip(singles, mols[name]):
                pkg.dfjk_build_J(hs.h, m["D"], m["J"])
                pkg.dfjk_build_K(hs.h, m["C"], m["C"].shape[1], None, m["K"])

        single = timed(loop, max(1, args.steps // 2))
        for hs in singles:
            hs.close()
        bt.close()
        res_d[name] = {"graph_ms": graph, "eager_ms": eager, "untuned_eager_ms": untuned,
                       "loop_of_single_builds_ms": single, "molecules_per_s": len(sizes) / graph * 1e3,
                       "k_tflops_aggregate": kfl / graph / 1e9, "j_bytes_gb": jbytes[name] / 1e9,
                       "tiles_by_bucket": tiles, "speedup_vs_loop": single / graph,
                       "speedup_vs_untuned": untuned / graph}
        if k16 is not None:
            res_d[name]["k16"] = k16
        log(name, res_d[name])
    res = {"metric": "DF-K TFLOP/s + J HBM GB/s vs FP64 plain; J/K builds to 1e-6 Eh",
           "value": res_d["f32"]["molecules_per_s"], "unit": "molecules/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": res_d["f32"]["graph_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"batched DF J/K: {len(sizes)} molecules, nao ~ U{{40..400}} "
                                  f"(sum {int(sizes.sum())}), naux = 4 nao, nocc = nao//5, one graph-captured "
                                  f"batched J+K per step", "nmol": int(len(sizes))},
           "f32": res_d["f32"], "bf16": res_d["bf16"]}
    print(json.dumps(res), flush=True)


def bench_c5(args):
    """Learned guess: train on the plain SCF's converged densities of
    n_train systems (nao=128, naux=512, nocc=24), then count J/K builds to
    1e-6 Eh on n_test held-out systems, learned guess against core guess."""
    import torch

    import paper_2506_06661_amd as pkg
    import synth
    from paper_2506_06661_amd import guess

    cfg = synth.C5
    b_scale = synth.C5_B_SCALE if args.b_scale is None else args.b_scale

    def system(seed):
        R, B, H = synth.scf_system(seed, cfg, b_scale)
        return pkg.Handle(torch.from_numpy(B).cuda(), cfg.nao), torch.from_numpy(H).cuda(), \
            torch.from_numpy(R).cuda()

    t0 = time.time()
    Xs, ts, nconv, scf_ms = [], [], 0, []
    for seed in range(args.n_train):
        h, H, R = system(seed)
        torch.cuda.synchronize()
        ts0 = time.perf_counter()
        recs, D, C = guess.run_scf(h, H, cfg.nocc)
        scf_ms.append((time.perf_counter() - ts0) * 1e3)
        if recs[-1][2]:
            nconv += 1
            _, Dc = guess.core_guess(h, H, cfg.nocc)
            Xs.append(guess.features(H, Dc, R))
            ts.append(guess.target(D, Dc))
        h.close()
        if seed % 200 == 0:
            log(f"  training data {seed}/{args.n_train}, {time.time() - t0:.0f} s")
    X = torch.cat(Xs).contiguous()
    t = torch.cat(ts).contiguous()
    mlp = pkg.MLP(8, 256, 65536)
    if args.mlp_bf16:
        mlp.set_compute(pkg.DFJK_BF16)
    tr = guess.Trainer(mlp, synth.uniform(1, synth.STREAM_MLP, mlp.nparam))
    torch.cuda.synchronize()
    tt = time.perf_counter()
    tr.fit(X, t, epochs=args.epochs, batch=65536, lr=1e-3,
           order_uniform=synth.uniform(2, synth.STREAM_MLP, X.shape[0] * args.epochs), log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - tt
    core, learned, proj, fb, fails, wrong, wrong_p = [], [], [], 0, 0, 0, 0
    for seed in range(2000, 2000 + args.n_test):
        h, H, R = system(seed)
        ref, _, _ = guess.run_scf(h, H, cfg.nocc)
        if not ref[-1][2]:
            fails += 1
            h.close()
            continue
        e_ref = ref[-1][0]
        core.append(guess.builds_to(ref, e_ref))
        out = guess.solve(h, tr, H, R, cfg.nocc)
        acc = guess.account(out, e_ref, ref)
        learned.append(acc["builds"])
        fb += out["fallback"]
        wrong += acc["wrong_state"]
        outp = guess.solve(h, tr, H, R, cfg.nocc, projected=True)
        accp = guess.account(outp, e_ref, ref)
        proj.append(accp["builds"])
        wrong_p += accp["wrong_state"]
        h.close()
    core, learned, proj = np.array(core, float), np.array(learned, float), np.array(proj, float)
    res = {"metric": "DF-K TFLOP/s + J HBM GB/s vs FP64 plain; J/K builds to 1e-6 Eh",
           "value": float(learned.mean()), "unit": "J/K builds to 1e-6 Eh (mean)", "n_gpus": 1,
           "steps": int(len(learned)), "warmup": 0, "ms_per_step": float(np.mean(scf_ms)),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64 SCF, " + ("bf16" if args.mlp_bf16 else "f32") + " MLP",
           "data": "synthetic",
           "config": {"workload": f"learned guess: nao={cfg.nao}, naux={cfg.naux}, nocc={cfg.nocc}, "
                                  f"{args.n_train} training systems, {args.n_test} held out, "
                                  f"B scaled by {b_scale}", "epochs": args.epochs, "b_scale": b_scale},
           "core_guess_builds_mean": float(core.mean()), "core_guess_builds_median": float(np.median(core)),
           "learned_builds_mean": float(learned.mean()), "learned_builds_median": float(np.median(learned)),
           "paired_mean_difference": float((learned - core).mean()),
           "projected_builds_mean": float(proj.mean()),
           "projected_paired_mean_difference": float((proj - core).mean()),
           "fallbacks": int(fb), "converged_to_other_state": int(wrong),
           "projected_converged_to_other_state": int(wrong_p),
           "test_systems_not_converged_plain": int(fails),
           "train_systems_converged": int(nconv), "train_pairs": int(X.shape[0]),
           "train_seconds": train_s, "plain_scf_ms_mean": float(np.mean(scf_ms))}
    print(json.dumps(res), flush=True)


def bench_c5mp(args):
    """Mixed-precision SCF on the SCF family (nao=128, naux=512, nocc=24):
    J/K from B stored in BF16 or FP16 until |FD - DF|_F < 1e-4, then from the
    FP64 B; J/K builds to 1e-6 Eh of the plain FP64 SCF on n_test systems."""
    import torch

    import paper_2506_06661_amd as pkg
    import synth
    from paper_2506_06661_amd import guess

    cfg = synth.C5
    b_scale = synth.C5_B_SCALE if args.b_scale is None else args.b_scale
    rows = {"plain": [], "bf16": [], "f16": []}
    fails = 0
    for seed in range(2000, 2000 + args.n_test):
        R, B, H = synth.scf_system(seed, cfg, b_scale)
        Bd = torch.from_numpy(B).cuda()
        Hd = torch.from_numpy(H).cuda()
        h64 = pkg.Handle(Bd, cfg.nao)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref, _, _ = guess.run_scf(h64, Hd, cfg.nocc)
        t_plain = (time.perf_counter() - t0) * 1e3
        if not ref[-1][2]:
            fails += 1
            h64.close()
            continue
        e_ref = ref[-1][0]
        rows["plain"].append((guess.builds_to(ref, e_ref), 0, t_plain, 0.0, 0.0))
        for name, code, tdt in [("bf16", pkg.DFJK_BF16, torch.bfloat16), ("f16", pkg.DFJK_F16, torch.float16)]:
            Bq = torch.empty(Bd.shape, dtype=tdt, device="cuda")
            pkg.dfjk_quantize(Bd, Bq, code, Bd.numel())
            hq = pkg.Handle(Bq, cfg.nao, dtype=code)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            recs, _, _ = guess.run_scf_mixed(hq, h64, Hd, cfg.nocc)
            ms = (time.perf_counter() - t0) * 1e3
            nlow = sum(1 for r in recs if r[3])
            n = guess.builds_to(recs, e_ref)
            low_err = [r[0] for r in recs if r[3]][-1] - e_ref
            rows[name].append((n if n is not None else float("nan"), nlow, ms, abs(recs[-1][0] - e_ref),
                               low_err))
            hq.close()
        h64.close()
        if (seed - 2000) % 50 == 0:
            log(f"  system {seed - 2000 + 1}/{args.n_test}")
    out = {}
    for name, r in rows.items():
        a = np.array(r, float)
        out[name] = {"builds_to_1e-6_mean": float(np.nanmean(a[:, 0])),
                     "builds_to_1e-6_median": float(np.nanmedian(a[:, 0])),
                     "not_reached": int(np.isnan(a[:, 0]).sum()),
                     "reduced_builds_mean": float(a[:, 1].mean()), "scf_ms_mean": float(a[:, 2].mean())}
        if name != "plain":
            out[name].update({"final_abs_err_max_Eh": float(a[:, 3].max()),
                              "reduced_phase_err_at_switch_median_Eh": float(np.median(a[:, 4])),
                              "reduced_phase_abs_err_at_switch_max_Eh": float(np.abs(a[:, 4]).max()),
                              "paired_builds_difference_mean": float(np.nanmean(a[:, 0] - np.array(
                                  rows["plain"], float)[:, 0]))})
    res = {"metric": "DF-K TFLOP/s + J HBM GB/s vs FP64 plain; J/K builds to 1e-6 Eh",
           "value": out["bf16"]["builds_to_1e-6_mean"], "unit": "J/K builds to 1e-6 Eh (mean, BF16 then FP64)",
           "n_gpus": 1, "steps": len(rows["plain"]), "warmup": 0, "ms_per_step": out["bf16"]["scf_ms_mean"],
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 SCF; J/K from bf16/f16 B, then f64 B", "data": "synthetic",
           "config": {"workload": f"mixed-precision SCF: nao={cfg.nao}, naux={cfg.naux}, nocc={cfg.nocc}, "
                                  f"{args.n_test} systems, B scaled by {b_scale}, switch at |FD-DF| < 1e-4",
                      "b_scale": b_scale},
           "plain": out["plain"], "bf16": out["bf16"], "f16": out["f16"],
           "plain_not_converged": fails}
    print(json.dumps(res), flush=True)


def bench_lrdf(args):
    """The long-range-DF shape: nao=1024 (the lattice of the nao=1024 workload),
    naux = 103 (about nao/10), nocc=200, FP64 B; one J and one K per step."""
    import torch

    import paper_2506_06661_amd as pkg
    import synth

    cfg = synth.C2
    naux = 103
    R = synth.positions(cfg)
    C = synth.C_occ(cfg.seed, cfg.nao, cfg.nocc)
    Bd = torch.from_numpy(synth.B_rows(cfg.seed, R, 0, naux)).cuda()
    Cd = torch.from_numpy(C).cuda()
    Dd = 2.0 * Cd @ Cd.T
    h = pkg.Handle(Bd, cfg.nao)
    lcfg = synth.Config("lrdf", cfg.nao, naux, cfg.nocc, cfg.seed)
    r = time_steps(pkg, h, Dd, Cd, lcfg, args.steps, args.warmup)
    h.close()
    ph = r["phase_ms"]
    g1, sy = k_flops(naux, cfg.nao, cfg.nocc)
    jbytes = 2.0 * naux * cfg.npair * 8
    res = {"metric": "DF-K TFLOP/s + J HBM GB/s vs FP64 plain; J/K builds to 1e-6 Eh",
           "value": (g1 + sy) / ph["K"] / 1e9, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"long-range DF shape: nao={cfg.nao}, naux={naux}, nocc={cfg.nocc}, FP64 B",
                      "nao": cfg.nao, "naux": naux, "nocc": cfg.nocc},
           "j_hbm_gbs": jbytes / ph["J"] / 1e6, "phase_ms": ph,
           "k_gemm1_tflops": g1 / ph["K_gemm1"] / 1e9, "k_syrk_tflops": sy / ph["K_syrk"] / 1e9}
    print(json.dumps(res), flush=True)


def bench_bform(args):
    """B = L^-1 Q at naux=4096 and 524800 columns (nao=1024 packed): the
    metric Cholesky and the forward substitution on the GPU, FP64."""
    import torch

    import paper_2506_06661_amd as pkg
    import synth

    cfg = synth.C2
    R = synth.positions(cfg)
    Q = torch.from_numpy(synth.B_full(cfg.seed, R, cfg.naux)).cuda()
    M = torch.from_numpy(synth.metric(cfg.seed, cfg.naux)).cuda()
    # Cholesky naux^3/3 flop, substitution naux^2 flop per column
    flops = cfg.naux ** 3 / 3.0 + float(cfg.naux) ** 2 * cfg.npair
    times = []
    for it in range(args.warmup + args.steps):
        Md, Qd = M.clone(), Q.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pkg.dfjk_form_B(cfg.naux, cfg.npair, Md, Qd, cfg.npair)
        torch.cuda.synchronize()
        if it >= args.warmup:
            times.append((time.perf_counter() - t0) * 1e3)
        del Md, Qd
    ms = float(np.median(times))
    res = {"metric": "DF-K TFLOP/s + J HBM GB/s vs FP64 plain; J/K builds to 1e-6 Eh",
           "value": flops / ms / 1e9, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"3-index factor B = L^-1 Q: naux={cfg.naux}, {cfg.npair} columns, "
                                  f"synthetic SPD metric, FP64 (Cholesky + forward substitution)",
                      "naux": cfg.naux, "ncol": cfg.npair},
           "flop_model": "naux^3/3 (Cholesky) + naux^2 * ncol (substitution)"}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "c5mp", "bform", "lrdf"],
                    help="c2: nao=1024 FP64 (+FP32) single builds (default); c3: nao=2048 BF16/FP16; "
                         "c4: 256-molecule batch; c5: learned-guess SCF experiment; "
                         "c5mp: mixed-precision SCF; bform: B = L^-1 Q on the GPU; "
                         "lrdf: naux = nao/10")
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--mlp-bf16", action="store_true",
                    help="c5: hidden-layer products of the network on the 16-bit matrix cores")
    ap.add_argument("--b-scale", type=float, default=None,
                    help="c5: scale of B in the SCF family (default: the generator's)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                           "COPY_WRITE_DIR"),
                    help="print the HBM traffic summary of four rocprofv3 --pmc output folders (no GPU)")
    ap.add_argument("--traffic-first", type=int, default=3,
                    help="dispatches per kernel that belong to the warm-up and timed steps")
    ap.add_argument("--traffic-command", default="",
                    help="the rocprofv3 commands, quoted into the summary")
    ap.add_argument("--cpu-rows", type=int, default=512,
                    help="aux rows in the CPU-oracle sample (0 = skip)")
    args = ap.parse_args()
    if args.traffic_summary:
        print(traffic_summary(*args.traffic_summary, args.traffic_first, args.traffic_command))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "c5mp":
        return bench_c5mp(args)
    if args.workload == "bform":
        return bench_bform(args)
    if args.workload == "lrdf":
        return bench_lrdf(args)
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
    # per-step events on the handle's stream (torch's current stream) around J and K
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    e0.record()
    for a, b, c in ev:
        a.record()
        pkg.dfjk_build_J(h.h, Dd, J)
        b.record()
        pkg.dfjk_build_K(h.h, Cd, cfg.nocc, None, K)
        c.record()
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    med = {"step": float(np.median([a.elapsed_time(c) for a, b, c in ev])),
           "J": float(np.median([a.elapsed_time(b) for a, b, c in ev])),
           "K": float(np.median([b.elapsed_time(c) for a, b, c in ev]))}
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
        "value": (g1_flops + sy_flops) / med["K"] / 1e9,
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
        "timing": f"value = algorithmic K flop / median of {args.steps} per-step K times (HIP events on the "
                  f"handle's stream); phase_ms and roofline = per-launch averages from the library's own events",
        "median_ms": med,
        "k_tflops_mean": (g1_flops + sy_flops) / k_ms / 1e9,
        "j_hbm_gbs": jbytes / med["J"] / 1e6,
        "jk_builds_per_s": 1000.0 / (total_ms / args.steps),
        "phase_ms": {"J": j_ms, "J_rho": jr_ms, "J_out": jo_ms, "K": k_ms, "K_gemm1": g1_ms,
                     "K_syrk": sy_ms, "K_finish": avg("K_finish")},
        "roofline": {
            "kernel": ("k_gemm1_f64" if args.dtype == "f64" else "k_gemm1_f32") + " (GEMM1 phase; the orbital "
                      "columns may be covered by two launches of different tiles)",
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
    # J with the DF diagonal from the same stream (sum_P B[P,p]^2)
    dg = torch.empty(cfg.npair, dtype=torch.float64, device="cuda")
    pkg.dfjk_build_J_diag(h.h, Dd, J, None, dg)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        pkg.dfjk_build_J_diag(h.h, Dd, J, None, dg)
    e1.record()
    torch.cuda.synchronize()
    jd_ms = e0.elapsed_time(e1) / args.steps
    res["j_with_df_diagonal"] = {"ms": jd_ms, "hbm_gbs": jbytes / jd_ms / 1e6,
                                 "overhead_vs_j": jd_ms / j_ms - 1.0}
    del dg
    # J for 8 densities through one pair of passes over B
    if dt_code == pkg.DFJK_F64:
        nd = 8
        Dm = Dd.unsqueeze(0).repeat(nd, 1, 1).contiguous()
        Jm = torch.empty_like(Dm)
        pkg.dfjk_build_J_multi(h.h, nd, Dm, Jm, None)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            pkg.dfjk_build_J_multi(h.h, nd, Dm, Jm, None)
        e1.record()
        torch.cuda.synchronize()
        jm_ms = e0.elapsed_time(e1) / args.steps
        res["j_8_densities"] = {"ms": jm_ms, "ms_per_density": jm_ms / nd, "speedup_vs_8_single": nd * j_ms / jm_ms,
                                "b_stream_gbs": jbytes / jm_ms / 1e6}
        del Dm, Jm
    # K of a second-order SCF trial density D = C_vir x C_occ^T + its
    # transpose, from the two factors (two GEMM1 passes + the full product)
    if dt_code == pkg.DFJK_F64:
        Cb = synth.C_occ(cfg.seed, cfg.nao, cfg.nao)
        x = synth.rotation(cfg.seed, cfg.nao - cfg.nocc, cfg.nocc)
        Ld = torch.from_numpy(np.ascontiguousarray(Cb[:, cfg.nocc:] @ x)).cuda()
        Rd = torch.from_numpy(np.ascontiguousarray(Cb[:, :cfg.nocc])).cuda()
        Kp = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
        pkg.dfjk_build_K_pair(h.h, Ld, Rd, cfg.nocc, 1, 1.0, Kp)
        torch.cuda.synchronize()
        pkg.dfjk_profile(h.h, max(args.steps, 1))
        e0.record()
        for _ in range(args.steps):
            pkg.dfjk_build_K_pair(h.h, Ld, Rd, cfg.nocc, 1, 1.0, Kp)
        e1.record()
        torch.cuda.synchronize()
        kp_ms = e0.elapsed_time(e1) / args.steps
        pp = pkg.dfjk_profile_read(h.h)
        pkg.dfjk_profile(h.h, 0)
        kp_g1 = pp["K_gemm1"][0] / max(pp["K_gemm1"][1], 1)
        kp_sy = pp["K_syrk"][0] / max(pp["K_syrk"][1], 1)
        kp_flops = 2 * g1_flops + 2 * sy_flops  # X_L and X_R; sum_P X_L X_R^T + X_R X_L^T (lower tiles)
        res["k_response_density"] = {
            "ms": kp_ms, "tflops": kp_flops / kp_ms / 1e9, "gemm1_ms": kp_g1, "gemm1_tflops": 2 * g1_flops / kp_g1 / 1e9,
            "gemm2_ms": kp_sy, "gemm2_tflops": 2 * sy_flops / kp_sy / 1e9, "ratio_to_k_occ": kp_ms / k_ms}
        del Ld, Rd, Kp
        # K of a general (here indefinite) density at this size: the two
        # factors (D, I), one call after a warm-up
        A = torch.from_numpy(synth.C_occ(cfg.seed + 1, cfg.nao, cfg.nao)).cuda()
        Dg = (A + A.T).contiguous()
        Kg = torch.empty((cfg.nao, cfg.nao), dtype=torch.float64, device="cuda")
        pkg.dfjk_build_K(h.h, None, 0, Dg, Kg)
        torch.cuda.synchronize()
        e0.record()
        pkg.dfjk_build_K(h.h, None, 0, Dg, Kg)
        e1.record()
        torch.cuda.synchronize()
        kd_ms = e0.elapsed_time(e1)
        kd_flops = 2 * 2.0 * cfg.naux * cfg.nao ** 3 + 2.0 * cfg.naux * cfg.nao * cfg.nao * (cfg.nao + 1)
        res["k_from_density"] = {"ms": kd_ms, "tflops": kd_flops / kd_ms / 1e9, "ratio_to_k_occ": kd_ms / k_ms,
                                 "form": "two factors (D, I): sum_P B_P D B_P"}
        del A, Dg, Kg
    res["measured_mfma_ceiling_tflops"] = {
        "f64_16x16x4": pkg.dfjk_probe_mfma(pkg.DFJK_F64), "f32_16x16x4": pkg.dfjk_probe_mfma(pkg.DFJK_F32),
        "bf16_32x32x16": pkg.dfjk_probe_mfma(pkg.DFJK_BF16)}
    hbm_read = pkg.dfjk_probe_hbm_read(Bd)
    res["measured_hbm_read_gbs"] = hbm_read
    res["j_frac_of_measured_hbm_read"] = res["j_hbm_gbs"] / hbm_read
    res["roofline"]["frac_of_measured_ceiling"] = (
        res["roofline"]["achieved"] / res["measured_mfma_ceiling_tflops"]["f64_16x16x4" if args.dtype == "f64"
                                                                         else "f32_16x16x4"])
    h.close()
    if args.dtype == "f64":
        # the same workload with B stored in FP32 (one RNE step from FP64)
        Bf = torch.empty(Bd.shape, dtype=torch.float32, device="cuda")
        pkg.dfjk_quantize(Bd, Bf, pkg.DFJK_F32, Bd.numel())
        h32 = pkg.Handle(Bf, cfg.nao, dtype=pkg.DFJK_F32)
        f32 = time_steps(pkg, h32, Dd, Cd, cfg, args.steps, args.warmup)
        g1_32 = f32["phase_ms"]["K_gemm1"]
        res["f32"] = {
            "k_tflops": (g1_flops + sy_flops) / f32["phase_ms"]["K"] / 1e9,
            "j_hbm_gbs": jbytes / 2 / f32["phase_ms"]["J"] / 1e6,
            "ms_per_step": f32["ms_per_step"], "phase_ms": f32["phase_ms"],
            "k_gemm1_frac_of_f32_peak": g1_flops / g1_32 / 1e9 / PEAK["f32"],
            "speedup_vs_f64_step": res["ms_per_step"] / f32["ms_per_step"],
        }
        h32.close()
        del Bf
    del Bd, Cd, Dd
    if args.cpu_rows > 0:
        log(f"timing the CPU oracle on {args.cpu_rows} aux rows ...")
        res["cpu_baseline"] = cpu_baseline(cfg, R, C, D, args.cpu_rows)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
