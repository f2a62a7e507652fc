"""Benchmark of the spin-adapted two-site DMRG hot path on one MI355X.

Workload (default): CAS(82,82), S=0, D=4096 multiplets, iron-sulfur-like
synthetic integrals, random mixed-canonical MPS with the two-site block at the
chain centre (sites 40, 41).  One step = the hot path at that block: H*psi in
the bulk precision (BF16 operands, FP32 accumulation) -- the Davidson matvec --
plus an FP64 H*psi of the same vector (the correction matvec), so every step
reports the mixed-precision throughput, the FP64 throughput and their
agreement.  Operator blocks are built once before timing (set-up, reported).

Prints one JSON line (see the fields below).  --gpus > 1 is not supported:
this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·ψ TFLOP/s & sweep time, CAS(82,82) D=4096, mixed vs FP64 at |ΔE|≤1e-6 Eh"
PEAK = {"bf16": 2500.0, "f32": 157.3, "f64": 78.6}  # dense MFMA TFLOP/s, MI355X


def workload(name):
    from synth.integrals import huckel_chain, iron_sulfur_like, small_cas
    if name == "cfg0":
        h, g, _ = small_cas(8, 0)
        return dict(name="CAS(8,8) S=0 D=64 centre two-site block", n=8, N=8, two_s=0, D=64, k=3, h=h, g=g, seed=0)
    if name == "cfg1":
        h, g, _ = huckel_chain(32, 1, naux=96)
        return dict(name="CAS(32,32) S=0 D=1024 centre two-site block, Hueckel-chain integrals", n=32, N=32,
                    two_s=0, D=1024, k=15, h=h, g=g, seed=1)
    if name == "cfg4":
        h, g, _ = iron_sulfur_like(4)
        return dict(name="CAS(82,82) S=0 D=4096 centre two-site block, Fe-S-like integrals", n=82, N=82, two_s=0,
                    D=4096, k=40, h=h, g=g, seed=4)
    raise SystemExit(f"unknown config {name}")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(lib_flops_fn):
    """The FP64 oracle (H_eff psi = V^T H V psi on explicit determinants) on a
    bounded sample: the centre H*psi of CAS(10,10), S=0, complete two-site
    space.  Reported as algorithmic TFLOP/s with the same flop count the GPU
    path uses for that H*psi."""
    from oracle import heff
    from synth.integrals import small_cas
    from synth.mps import random_mps, random_psi
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    h, g, _ = small_cas(10, 21)
    mps = random_mps(10, 10, 0, 1000, k=4, seed=21)
    psi, lay = random_psi(mps)
    flops = lib_flops_fn(h, g, mps, psi)
    he = heff.HeffDefinition(h, g, mps, lay)
    he.apply(psi)  # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        he.apply(psi)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 5:
            break
    dt = (time.perf_counter() - t0) / reps
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"centre H*psi of CAS(10,10) S=0 (complete two-site space, {psi.size} coefficients), "
                      f"{reps} reps after 1 warm-up, {dt * 1e3:.0f} ms each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default=os.environ.get("DMRG_BENCH_CONFIG", "cfg4"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    from paper_2503_20700_amd.binding import BF16, DMRG, FP64
    from synth.mps import random_mps, random_psi

    w = workload(args.config)
    t0 = time.perf_counter()
    mps = random_mps(w["n"], w["N"], w["two_s"], w["D"], k=w["k"], seed=w["seed"])
    psi, lay = random_psi(mps, seed=w["seed"] + 1)
    log(f"{w['name']}: MPS drawn in {time.perf_counter() - t0:.1f}s, psi has {psi.size} coefficients")
    dm = DMRG(w["h"], w["g"], w["N"], w["two_s"])
    bs, cnt = mps.bond_table()
    t0 = time.perf_counter()
    dm.set_mps(w["k"], bs, cnt, mps.site_blocks_flat())
    t_env = time.perf_counter() - t0
    log(f"operator blocks built in {t_env:.1f}s")
    t0 = time.perf_counter()
    y64, flops = dm.hpsi(psi, FP64)   # plans the H*psi task lists, first FP64 matvec
    t_plan = time.perf_counter() - t0
    st = dm.stats()
    log(f"H*psi planned ({st['n_terms']} terms, {st['n_tasks']} block products, {flops:.3e} flop) in {t_plan:.1f}s")

    def step():
        ylo, _ = dm.hpsi(psi, BF16)
        y, _ = dm.hpsi(psi, FP64)
        return ylo, y

    for i in range(args.warmup):
        step()
        log(f"warm-up {i + 1}/{args.warmup} done")
    # timed region: BF16 and FP64 matvecs, with device-event timing of every GEMM launch
    t_lo = t_hi = 0.0
    n_lo = n_hi = 0
    t_start = time.perf_counter()
    for i in range(args.steps):
        dm.kernel_timing(1)
        ylo, _ = dm.hpsi(psi, BF16)
        ms, nl = dm.kernel_timing(0)
        t_lo += ms
        n_lo += nl
        dm.kernel_timing(1)
        y, _ = dm.hpsi(psi, FP64)
        ms, nl = dm.kernel_timing(0)
        t_hi += ms
        n_hi += nl
        log(f"step {i + 1}/{args.steps}: bf16 {t_lo / (i + 1):.1f} ms, fp64 {t_hi / (i + 1):.1f} ms of kernels")
    t_wall = time.perf_counter() - t_start
    ms_step = t_wall / args.steps * 1e3
    lo_tflops = flops * args.steps / (t_lo * 1e-3) / 1e12
    hi_tflops = flops * args.steps / (t_hi * 1e-3) / 1e12
    rel = float(np.abs(ylo - y).max() / np.abs(y).max())
    e_lo, e_hi = float(psi @ ylo), float(psi @ y)

    base = None
    if not args.no_cpu_baseline:
        def fl(h, g, m, p):
            d = DMRG(h, g, m.n_elec, m.two_s)
            b, c = m.bond_table()
            d.set_mps(m.k, b, c, m.site_blocks_flat())
            _, f = d.hpsi(p, FP64)
            d.close()
            return f
        log("timing the oracle on its bounded sample")
        base = cpu_baseline(fl)

    out = {
        "metric": METRIC,
        "value": lo_tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": w["name"], "n_orb": w["n"], "n_elec": w["N"], "two_s": w["two_s"], "D": w["D"],
                   "two_site_block": [w["k"], w["k"] + 1], "psi_len": int(psi.size)},
        "roofline": {"bound": "mfma", "achieved": lo_tflops, "peak": PEAK["bf16"], "unit": "TFLOP/s",
                     "frac": lo_tflops / PEAK["bf16"], "traffic": None},
        "cpu_baseline": base,
        "hpsi_flops": flops,
        "fp64": {"tflops": hi_tflops, "roofline_frac": hi_tflops / PEAK["f64"], "ms_per_hpsi": t_hi / args.steps},
        "bf16": {"ms_per_hpsi": t_lo / args.steps, "launches_per_hpsi": n_lo // max(args.steps, 1)},
        "speedup_bf16_vs_fp64": t_hi / t_lo if t_lo > 0 else None,
        "rel_err_bf16_vs_fp64": rel,
        "rayleigh_bf16_minus_fp64_Eh": e_lo - e_hi,
        "setup_s": {"operator_blocks": t_env, "hpsi_plan": t_plan},
        "op_bytes_f64": st["op_bytes"],
        "peak_device_bytes": st["peak_bytes"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
