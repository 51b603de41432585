"""Times the FP64 oracle on the benchmark workloads: the CPU baseline of the estimator.

TEST INFRASTRUCTURE: this times the oracle (the plain CPU implementation of the
estimator that the tests use); the library never runs it.

For each workload the polygon counts (the estimator on unit shells, Appendix A) and the
forward pass (shell fields, product sums, normalisation; Sec. 2) are timed separately,
best of --repeat runs, and for the gradient workload also the FP64 gradient.  The
thread count (SciPy FFT workers and BLAS threads) is set by --cores before NumPy loads.

Usage: python -m oracle.timing --cores 8 --repeat 3 --workloads bispec_64,bispec_256_lognormal --out t.json
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time


def _set_threads(cores: int) -> int:
    """Pins the process to `cores` CPUs and sets the BLAS thread count (before NumPy loads)."""
    avail = sorted(os.sched_getaffinity(0))
    cores = max(1, min(cores, len(avail)))
    os.sched_setaffinity(0, set(avail[:cores]))
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        os.environ[var] = str(cores)
    return cores


def _best(fn, repeat):
    best, out = float("inf"), None
    for _ in range(repeat):
        t0 = time.perf_counter()
        out = fn()
        best = min(best, time.perf_counter() - t0)
    return best, out


def time_workload(name: str, repeat: int) -> dict:
    import numpy as np

    import fieldgen
    import oracle as O
    w = fieldgen.WORKLOADS[name]
    N, order, nb, width = w["N"], w["order"], w["n_shells"], w["width"]
    fields = fieldgen.workload_fields(name, dtype=np.float32).astype(np.float64)
    cand = O.candidate_tuples(order, nb, O.is_alias_free(N, order, nb, width))
    t_counts, counts = _best(lambda: O.polygon_counts(N, order, nb, width, cand), repeat)
    keep = counts > 0
    rec = {"workload": name, "N": N, "order": order, "n_shells": nb, "width": width, "batch": len(fields),
           "n_closing": int(keep.sum()), "counts_s": t_counts}

    def forward():
        return [O.polyspectrum(f, order, nb, width, counts=counts, return_fields=bool(w.get("target_seed")))
                for f in fields]

    t_fwd, res = _best(forward, repeat)
    rec["forward_s"] = t_fwd
    G = N ** 3
    rec["forward_rate"] = rec["n_closing"] * G * len(fields) / t_fwd
    if w.get("target_seed") is not None:
        target = O.polyspectrum(fieldgen.gaussian_field(N, w["target_seed"]).astype(np.float32).astype(np.float64),
                                order, nb, width, counts=counts)["B"]

        def backward():
            return [O.gradient(f, order, nb, width, 2.0 * (r["B"] - target), result=r) for f, r in zip(fields, res)]

        rec["gradient_s"], _ = _best(backward, repeat)
        rec["forward_backward_rate"] = rec["n_closing"] * G * len(fields) / (t_fwd + rec["gradient_s"])
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--cores", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--repeat", type=int, default=3)
    ap.add_argument("--workloads", default="bispec_64,bispec_256_lognormal,trispec_256_lognormal,bispec_grad_128x8")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    cores = _set_threads(args.cores)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    out = {"cores": cores, "cpu": cpu or platform.processor(), "repeat": args.repeat, "kind": "oracle", "results": []}
    for name in args.workloads.split(","):
        print(f"[timing] {name} on {cores} cores", file=sys.stderr, flush=True)
        out["results"].append(time_workload(name, args.repeat))
        print(json.dumps(out["results"][-1]), file=sys.stderr, flush=True)
    text = json.dumps(out, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    print(text)


if __name__ == "__main__":
    main()
