#!/usr/bin/env python3
"""Bispectrum forward + backward on one MI355X: 512^3 lognormal field, 64 unit-width shells.

One step = the whole hot path on one field resident in HBM: input transform,
64 shell fields, the matrix-core product sums with float64 reduction and
normalisation, and the adjoint back to dL/d delta (loss sum_t B_t^2, so
dL/dB = 2 B).  Polygon counts are computed once when the plan is built and are
not part of a step.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bispec_512_lognormal")
    ap.add_argument("--precision", default="fp16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--bwd-precision", default="auto", choices=["auto", "bf16", "fp16", "fp32"],
                    help="the adjoint's arithmetic; auto: the BF16 split after a split-precision forward "
                         "(the matrix cores sustain a higher rate on BF16 operands under the power limit), "
                         "FP32 after FP32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-compare", action="store_true")
    ap.add_argument("--cpu-planes", type=int, default=8, help="x0-planes in the oracle's timing sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (reference for HBM counters)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    """Hash of the sources of the matrix-core kernels (the contraction and the adjoint)."""
    h = hashlib.sha256()
    for f in ("contract_tiles.h", "contract_tiles_lo.hip", "contract_tiles_hi.hip", "contract_j3.hip",
              "adjoint.h", "adjoint.hip", "adjoint_fp32.hip", "adjoint_bf16.hip", "adjoint_fp16.hip",
              "mfma_ops.h", "fft_core.h", "common.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1904_11055_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch of a kernel from committed counter runs, if still current."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def adjoint_weight_entries(tuples) -> int:
    """Distinct adjoint weights (m, sorted rest of t without one position of m): each
    closing tuple t feeds a_m for every position of m with the product of the others."""
    seen = set()
    for t in tuples.tolist():
        for p in range(len(t)):
            seen.add((t[p],) + tuple(sorted(t[:p] + t[p + 1:])))
    return len(seen)


def roofline(kernel: str, ms: float, alg_flops: float, issued_flops: float, peak: float, traffic):
    """achieved/frac use algorithmic flops; issued_* count every matrix-core product launched."""
    achieved = alg_flops / (ms * 1e-3) / 1e12
    issued = issued_flops / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "kernel": kernel,
            "alg_flops_per_launch": alg_flops, "ms_per_launch": ms,
            "issued_flops_per_launch": issued_flops, "issued_tflops": issued, "issued_frac": issued / peak}


def cpu_baseline(delta32, w, n_closing, planes: int):
    """The FP64 oracle timed on a bounded sample of the same workload, scaled to a full step.

    Sample: one full-grid inverse real FFT and one forward real FFT (each needed
    n_shells + 1 times per step), plus the per-grid-point work (pair products, the
    product-sum matrix product and the adjoint's weighted pair sum) over `planes`
    x0-planes of the grid, scaled by N / planes.
    """
    import numpy as np

    import oracle as O
    from oracle.polyspec import irfftn, rfftn
    N, nb, width = w["N"], w["n_shells"], w["width"]
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    delta = delta32.astype(np.float64)
    t0 = time.perf_counter()
    dhat = rfftn(delta)
    t_r2c = time.perf_counter() - t0
    t0 = time.perf_counter()
    _ = irfftn(dhat, s=(N, N, N))
    t_c2r = time.perf_counter() - t0
    pl = list(range(planes))
    fields = O.shell_fields_on_planes(dhat, N, nb, width, pl)          # [nb, planes, N, N]
    tuples = O.candidate_tuples(3, nb, O.is_alias_free(N, 3, nb, width))
    t0 = time.perf_counter()
    S = O.product_sums(fields, tuples)
    t_ctr = time.perf_counter() - t0
    wts = np.linspace(-1.0, 1.0, len(tuples))
    t0 = time.perf_counter()
    W = O.adjoint_weights(tuples, wts, nb)
    pairs = O.pair_list(nb)
    flat = fields.reshape(nb, -1)
    a = np.empty_like(flat)
    for x0 in range(0, flat.shape[1], 8192):
        blk = flat[:, x0:x0 + 8192]
        a[:, x0:x0 + 8192] = W @ (blk[pairs[:, 0] - 1] * blk[pairs[:, 1] - 1])
    t_adj = time.perf_counter() - t0
    del S, a
    scale = N / planes
    t_step = (nb + 1) * (t_r2c + t_c2r) + scale * (t_ctr + t_adj)
    G = N ** 3
    return {
        "value": n_closing * G / t_step,
        "unit": "bin-triplets*gridpts/s",
        "cores": cores,
        "kind": "oracle",
        "extrapolated": True,
        "sample": (f"FP64 oracle: one {N}^3 rfftn ({t_r2c:.2f} s) and irfftn ({t_c2r:.2f} s) scaled x{nb + 1} "
                   f"each; product sums over all {len(tuples)} candidate triplets and the adjoint pair "
                   f"GEMM on {planes} of {N} x0-planes ({t_ctr:.2f} s + {t_adj:.2f} s) scaled x{scale:g}; "
                   f"estimated (extrapolated) step {t_step:.1f} s"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the grid would shard "
              "over x0-slabs with one small all-reduce per direction).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 4, "copies": 3}), flush=True)
        return

    import fieldgen
    import paper_1904_11055_amd as ps

    w = fieldgen.WORKLOADS[args.workload]
    order = w["order"]
    if order not in (3, 4, 5, 6):
        raise SystemExit("the benchmark step needs an order-3 to order-6 workload")
    # orders 3 and 4 (up to 64 shells) have the adjoint: a step is forward +
    # backward; otherwise forward only
    streamed = bool(w.get("stream"))
    N, nb, width, batch = w["N"], w["n_shells"], w["width"], len(w["seeds"])
    has_backward = order in (3, 4) and nb <= 64
    codes = {"bf16": ps.SPLIT_BF16, "fp16": ps.SPLIT_FP16, "fp32": ps.FP32}
    prec = codes[args.precision]
    bwd_name = args.bwd_precision if args.bwd_precision != "auto" else ("fp32" if args.precision == "fp32" else "bf16")
    bwd_code = codes[bwd_name]
    dev = torch.device("cuda:0")
    flags = ps.STREAM_SLABS if streamed else 0
    if w.get("spectrum_of"):
        # the band-limited interpolation of a smaller workload's field (input preparation,
        # outside the timed steps)
        log(f"generating the {w['spectrum_of']} field and its {N}^3 interpolation")
        fields = fieldgen.workload_fields(w["spectrum_of"], dtype=np.float32)
        kc = int(np.ceil((nb + 0.5) * width)) - 1
        # the inverse transform on the host (a threaded pocketfft through SciPy), so that
        # preparing the input launches no GPU work besides the copy
        import scipy.fft
        hs = fieldgen.zero_padded_half_spectrum(fields[0], N, kc)
        xr = scipy.fft.irfftn(hs, s=(N, N, N), workers=min(16, os.cpu_count() or 1))
        del hs
        x = torch.from_numpy(np.ascontiguousarray(xr, dtype=np.float32))[None].to(dev)
        del xr
    else:
        log(f"generating {args.workload} fields")
        fields = fieldgen.workload_fields(args.workload, dtype=np.float32)
        x = torch.from_numpy(fields).to(dev)
    torch.cuda.synchronize()
    log("building plan (float64 polygon counts)")
    t0 = time.perf_counter()
    plan = ps.Plan(N, order, nb, width, batch=batch, precision=prec, flags=flags, device=dev)
    launches = N // plan.slab_planes      # contraction launches per step (slabs when streamed)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    log(f"plan built in {plan_s:.2f} s: {plan.n_closing} closing tuples")
    G = N ** 3

    def step():
        plan.shells(x)
        B = plan.contract()
        if not has_backward:
            return B, None
        if bwd_code != prec:          # the adjoint's precision, set between the calls
            plan.precision = bwd_code
        g = plan.backward(2.0 * B)
        if bwd_code != prec:
            plan.precision = prec
        return B, g

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ps.polyspec_profile(plan.handle, True)
    ps.polyspec_profile_read(plan.handle)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B, g = step()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    prof = ps.polyspec_profile_read(plan.handle)
    ms_step = 1000.0 * t / args.steps
    log(f"timed {args.steps} steps: {ms_step:.2f} ms/step")

    def avg(name):
        ms, n = prof[name]
        return ms / n if n else 0.0

    fwd = ["input_q3", "input_q2", "input_q1", "shell_p1", "shell_p2", "shell_p3", "contract", "reduce", "gather"]
    bwd = ["adj_weights", "adj_gemm", "adj_q3", "adj_q2", "adj_q1", "grad_p1", "grad_p2", "grad_p3"]
    def per_step(name):   # a streamed step launches the slab kernels once per slab
        return prof[name][0] / args.steps

    fwd_ms = sum(per_step(k) for k in fwd)
    bwd_ms = sum(per_step(k) for k in bwd)
    ctr_ms = avg("contract")
    adj_ms = avg("adj_gemm")
    n_pairs = nb * (nb + 1) // 2
    n_triples = nb * (nb + 1) * (nb + 2) // 6
    n_rests = n_pairs if order == 3 else n_triples   # products the adjoint forms
    peak = PEAK_TFLOPS[args.precision]
    # algorithmic flops per launch: 2 per (closing triplet x point) + 1 per (pair x point)
    # for the contraction; 2 per (adjoint weight x point) + 1 per (pair x point) for the
    # adjoint product, whatever the tiles the kernels actually issue
    # the FP16 split of an order-3 plan runs the shell-block aligned kernel
    ctr_kernel = "contract_j3" if (args.precision == "fp16" and order == 3 and nb <= 64) else "contract_tiles"
    # algorithmic flops: 2 per (closing tuple x point), plus the row products formed once
    # per point: 1 per pair (orders 3 to 5) and 2 per triple (orders 5 and 6)
    row_flops = (n_pairs if order <= 5 else 0) + (2 * n_triples if order >= 5 else 0)
    ctr_roof = roofline(ctr_kernel, ctr_ms, (2.0 * plan.n_closing + row_flops) * G * batch / launches,
                        ps.polyspec_issued_flops(plan.handle, "contract") / launches, peak,
                        load_traffic(ctr_kernel, args.workload, args.precision))
    if has_backward:
        n_w = adjoint_weight_entries(plan.tuples)
        adj_kernel = "adjoint_gemm" if order == 3 else "adjoint4_gemm"
        plan.precision = bwd_code         # the issued products of the adjoint's own precision
        adj_issued = ps.polyspec_issued_flops(plan.handle, "adj_gemm")
        plan.precision = prec
        adj_roof = roofline(adj_kernel, adj_ms,
                            (2.0 * n_w + n_rests * (order - 2)) * G * batch / launches,
                            adj_issued / launches, PEAK_TFLOPS[bwd_name],
                            load_traffic(adj_kernel, args.workload, bwd_name))
        dominant, other = (adj_roof, ctr_roof) if adj_ms >= ctr_ms else (ctr_roof, adj_roof)
    else:
        n_w, dominant, other = None, ctr_roof, None
    # a streamed plan's FP16 mode takes the BF16 split in the adjoint (its field scales are
    # per slab)
    bwd_prec = (("bf16" if (streamed and bwd_name == "fp16") else bwd_name) if has_backward else None)
    dtype_label = args.precision if bwd_prec in (None, args.precision) else f"{args.precision} fwd / {bwd_prec} bwd"
    names = {3: ("bispectrum", "bin-triplets"), 4: ("trispectrum", "bin-quadruples"),
             5: ("quadspectrum", "bin-quintuples"), 6: ("pentaspectrum", "bin-sextuples")}[order]
    out = {
        "metric": ("bispectrum bin-triplets*gridpts/s at 512^3 (split-MFMA vs FP32); fwd+bwd ms"
                   if (order == 3 and N == 512 and has_backward)
                   else f"{names[0]} {names[1]}*gridpts/s at {N}^3 (split-MFMA"
                        + (", streamed slabs" if streamed else "") + "); "
                        + ("fwd+bwd ms" if has_backward else "fwd ms")),
        "value": plan.n_closing * G * batch / (ms_step * 1e-3),
        "unit": f"{names[1]}*gridpts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_label, "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "order": order, "n_shells": nb, "shell_width": width,
                   "batch": batch, "field": w["field"], "seeds": w["seeds"], "n_closing": plan.n_closing,
                   "precision": args.precision, "parallelism": "none (1 GPU)"},
        "fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "plan_s": plan_s,
        "contract_ms": ctr_ms * launches,
        "contract_rate": plan.n_closing * G * batch / (ctr_ms * launches * 1e-3),
        "phase_ms": {k: round(avg(k), 4) for k in ps.PHASES if prof[k][1]},   # per launch
        "launches_per_step": {k: prof[k][1] // args.steps for k in ps.PHASES if prof[k][1]},
        "roofline": dominant,
        "roofline_other": other,
        "adjoint_weights": n_w,
    }
    if not args.no_fp32_compare and args.precision != "fp32":
        plan.precision = ps.FP32
        plan.contract()
        ps.polyspec_profile_read(plan.handle)
        for _ in range(2):
            plan.contract()
        p32 = ps.polyspec_profile_read(plan.handle)
        ms32 = p32["contract"][0] / max(1, p32["contract"][1])
        out["fp32_contract_ms"] = ms32 * launches
        out["fp32_contract_rate"] = plan.n_closing * G * batch / (ms32 * launches * 1e-3)
        out["split_speedup_vs_fp32"] = ms32 / ctr_ms
        plan.precision = prec
        log(f"fp32 contraction {ms32:.2f} ms vs {args.precision} {ctr_ms:.2f} ms")
    plan.close()
    del x
    torch.cuda.empty_cache()
    if streamed:
        out["config"]["streamed_slab_planes"] = plan.slab_planes
        out["config"]["input"] = f"{w['spectrum_of']} field interpolated (band-limited) to {N}^3"
    if not args.no_cpu_baseline and order == 3 and not w.get("spectrum_of"):
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(fields[0], w, plan.n_closing * batch, args.cpu_planes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
