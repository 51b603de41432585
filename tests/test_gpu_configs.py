"""GPU parity at the full sizes of the benchmark workloads, in the benchmark's launch configuration.

* 256^3 bispectrum, 40 shells of width 2: every closing triplet against the FP64 oracle
  (counts bit-exact, B to the precision's tolerance, per-tuple error relative to the
  term magnitude A_t = sum_x |d_i d_j d_k| / (N^3 n_t)).
* The 512^3 benchmark's 64 unit shells on a 256^3 lognormal field (alias-free: 3 x 64.5 <=
  256): every closing triplet against the oracle in all three precisions, and the gradient
  of a random linear loss against the oracle gradient over the whole grid.  This exercises
  every wave, slot and tile of the order-3 contraction and every block of the adjoint at
  the benchmark's shell count.
* 512^3 itself: every count against the stored table (alias-free counts do not depend on
  N), the pair-sum rule, B of every closing triplet over a shell sample that reaches every
  wave (j mod 8) and every shell block, and the gradient of a loss supported on that
  sample's triplets against the oracle gradient (which then needs only the sample's fields).
* 256^3 trispectrum (24 shells of width 2), orders 5 and 6, the 128^3 x 8 gradient batch
  and the streamed 1024^3 plan as described at each test.
Measured errors are printed (and appended to $POLYSPEC_ERROR_LOG when it is set).
"""
import itertools
import os
import sys

import numpy as np
import pytest

import fieldgen
import oracle as O
from conftest import PRECISION_NAMES, record_error

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(msg):
    print(f"[configs] {msg}", file=sys.stderr, flush=True)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _gpu_run(fields, order, nb, width, precision, flags=0):
    import torch
    import paper_1904_11055_amd as ps
    plan = ps.Plan(fields.shape[-1], order, nb, width, batch=fields.shape[0], precision=precision,
                   flags=flags, device="cuda:0")
    plan.shells(torch.from_numpy(fields).to("cuda:0"))
    B = plan.contract().cpu().numpy()
    bins, quot = plan.candidates()
    return plan, B, bins, quot


def _pair_sum_check(tuples, counts, N, nb, width):
    table = {tuple(int(v) for v in t): int(c) for t, c in zip(tuples, counts)}
    S = O.shell_mode_counts(N, nb, width)
    n = 0
    for i in range(1, nb + 1):
        for j in range(i, nb + 1):
            if i + j + 1 > nb:
                continue
            tot = sum(table.get(tuple(sorted((i, j, k))), 0) for k in range(1, nb + 1))
            assert tot == S[i - 1] * S[j - 1] - (S[i - 1] if i == j else 0), (i, j)
            n += 1
    assert n > 0


_CACHE = {}


def _fields_cached(name):
    key = ("fields", name)
    if key not in _CACHE:
        _CACHE[key] = fieldgen.workload_fields(name)
    return _CACHE[key]


def _golden_64shell_counts():
    """Closing triplets and counts of 64 unit-width shells (any alias-free grid)."""
    if "g64" not in _CACHE:
        a = np.loadtxt(os.path.join(GOLDEN, "bispec_64shells_counts.txt.gz"), dtype=np.int64)
        _CACHE["g64"] = (a[:, :3], a[:, 3])
    return _CACHE["g64"]


def _candidate_counts(cand, tuples, counts):
    """Counts for every candidate from a closing table (0 where the candidate does not close)."""
    table = {tuple(int(v) for v in t): int(c) for t, c in zip(tuples, counts)}
    return np.array([table.get(tuple(int(v) for v in t), 0) for t in cand], dtype=np.int64)


def _integral(quot):
    """Every count quotient within max(1e-3, |q| 2^-46) of an integer (the plan's own bound)."""
    q = np.asarray(quot, dtype=np.float64)
    return bool(np.all(np.abs(q - np.rint(q)) < np.maximum(1e-3, np.ldexp(np.abs(q), -46))))


def _sample(plan_tuples, shells):
    allowed = set(shells)
    return [tuple(int(v) for v in t) for t in plan_tuples if set(int(v) for v in t) <= allowed]


def _subset_sums(fields, shells, tuples, absolute=False):
    """S_t (or sum_x |prod d|) over tuples whose shells all lie in `shells`, from the oracle's
    product sums on those fields alone (the shells renumbered 1..len(shells))."""
    pos = {s: n + 1 for n, s in enumerate(shells)}
    t = np.array([[pos[v] for v in tt] for tt in tuples], dtype=np.int64)
    return O.product_sums(np.abs(fields) if absolute else fields, t)


def _magnitudes(fields, tuples, counts, N, every=1):
    """A_t = sum_x |prod_j d_{t_j}| / (N^3 n_t); with every > 1 estimated from every `every`-th x0-plane."""
    sub = fields[:, ::every] if every > 1 else fields
    return every * O.product_sums(np.abs(sub), tuples) / (float(N) ** 3 * np.asarray(counts))


# ---------------------------------------------------------------------------------------
# 256^3 bispectrum, 40 shells of width 2: every closing triplet
# ---------------------------------------------------------------------------------------
def _c2_reference():
    if "c2" not in _CACHE:
        w = fieldgen.WORKLOADS["bispec_256_lognormal"]
        delta = _fields_cached("bispec_256_lognormal")[0].astype(np.float64)
        say("oracle: 256^3, 40 shells of width 2 (counts, every triplet)")
        ref = O.polyspectrum(delta, 3, w["n_shells"], w["width"], return_fields=True)
        say("oracle: term magnitudes (every 4th x0-plane)")
        ref["A"] = _magnitudes(ref["fields"], ref["tuples"], ref["counts"], w["N"], every=4)
        del ref["fields"]
        _CACHE["c2"] = ref
    return _CACHE["c2"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_bispec_256_lognormal(gpu, precision, tol):
    w = fieldgen.WORKLOADS["bispec_256_lognormal"]
    fields = _fields_cached("bispec_256_lognormal")
    ref = _c2_reference()
    plan, B, bins, quot = _gpu_run(fields, 3, w["n_shells"], w["width"], precision)
    assert _integral(quot)
    assert np.array_equal(plan.tuples, ref["tuples"])
    assert np.array_equal(plan.counts, ref["counts"])
    _pair_sum_check(plan.tuples, plan.counts, w["N"], w["n_shells"], w["width"])
    rel = _rel(B[0], ref["B"])
    scaled = float(np.max(np.abs(B[0] - ref["B"]) / ref["A"]))
    record_error("256^3 bispectrum, 40 shells of width 2 (lognormal)", PRECISION_NAMES[precision],
                 n_tuples=len(ref["B"]), rel_l2=rel, max_scaled=scaled)
    assert rel < tol
    assert scaled < tol
    plan.close()


# ---------------------------------------------------------------------------------------
# The benchmark's 64 unit shells on 256^3: every triplet and the whole gradient
# ---------------------------------------------------------------------------------------
def _c5_shells_256_reference():
    if "c5_256" not in _CACHE:
        N, nb = 256, 64
        delta = _fields_cached("bispec_256_lognormal")[0].astype(np.float64)
        tuples, counts = _golden_64shell_counts()
        cand = O.candidate_tuples(3, nb, True)
        say("oracle: 256^3 with 64 unit shells (every triplet, then the gradient)")
        ref = O.polyspectrum(delta, 3, nb, 1.0, counts=_candidate_counts(cand, tuples, counts),
                             return_fields=True)
        assert np.array_equal(ref["tuples"], tuples)
        say("oracle: term magnitudes (every 4th x0-plane)")
        ref["A"] = _magnitudes(ref["fields"], ref["tuples"], ref["counts"], N, every=4)
        say("oracle: gradient over the whole 256^3 grid")
        g = np.random.default_rng(55).standard_normal(len(ref["B"]))
        g_hat = O.gradient_spectrum(N, 3, nb, 1.0, ref["tuples"], ref["counts"], ref["fields"], g)
        ref["g"] = g
        ref["grad"] = O.polyspec.irfftn(g_hat, s=(N, N, N)) * float(N) ** 3
        del ref["fields"], g_hat
        _CACHE["c5_256"] = ref
    return _CACHE["c5_256"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_bispec_64_unit_shells_256_every_tuple_and_gradient(gpu, precision, tol):
    import torch
    import paper_1904_11055_amd as ps
    fields = _fields_cached("bispec_256_lognormal")
    ref = _c5_shells_256_reference()
    plan = ps.Plan(256, 3, 64, 1.0, precision=precision, device="cuda:0")
    assert np.array_equal(plan.tuples, ref["tuples"]) and np.array_equal(plan.counts, ref["counts"])
    x = torch.from_numpy(fields).to("cuda:0").requires_grad_(True)
    Bt = ps.polyspectrum(x, plan)
    B = Bt.detach().cpu().numpy()[0]
    Bt.backward(torch.from_numpy(ref["g"])[None].to("cuda:0"))
    grad = x.grad.cpu().numpy()[0]
    rel = _rel(B, ref["B"])
    scaled = float(np.max(np.abs(B - ref["B"]) / ref["A"]))
    grel = _rel(grad, ref["grad"])
    record_error("256^3, the 512^3 benchmark's 64 unit shells (lognormal)", PRECISION_NAMES[precision],
                 n_tuples=len(B), rel_l2=rel, max_scaled=scaled, grad_rel_l2=grel)
    assert rel < tol
    assert scaled < tol
    assert grel < 1e-4
    plan.close()


# ---------------------------------------------------------------------------------------
# 512^3, 64 unit shells: the benchmark's plan
# ---------------------------------------------------------------------------------------
# Shells (1-based) whose j - 1 covers every residue mod 8 (the wave of the order-3
# contraction), every slot j // 8 and every 16-shell block.
SHELLS_512 = [1, 2, 11, 20, 29, 30, 39, 47, 48, 56, 63, 64]


def _c5_sample_reference(order_check=True):
    if "c5_512" not in _CACHE:
        N, nb = 512, 64
        delta = _fields_cached("bispec_512_lognormal")[0].astype(np.float64)
        tuples, counts = _golden_64shell_counts()
        sample = _sample(tuples, SHELLS_512)
        idx = {tuple(int(v) for v in t): n for n, t in enumerate(tuples)}
        sel = np.array([idx[t] for t in sample])
        say(f"oracle: 512^3 fields of {len(SHELLS_512)} shells, {len(sample)} triplets")
        dhat = O.polyspec.rfftn(delta)
        d = O.shell_fields_from_hat(dhat, N, nb, 1.0, SHELLS_512)
        del dhat
        n_t = counts[sel]
        say("oracle: 512^3 product sums of the sample")
        S = _subset_sums(d, SHELLS_512, sample)
        A = 2 * _subset_sums(d[:, ::2], SHELLS_512, sample, absolute=True) / (float(N) ** 3 * n_t)
        # gradient of L = sum_t g_t B_t with g supported on the sample's triplets
        g = np.zeros(len(tuples))
        g[sel] = np.random.default_rng(56).standard_normal(len(sel))
        say("oracle: 512^3 gradient from the sample's fields")
        g_hat = O.gradient_spectrum(N, 3, nb, 1.0, tuples, counts, d, g, shells=SHELLS_512)
        del d
        grad = O.polyspec.irfftn(g_hat, s=(N, N, N)) * float(N) ** 3
        del g_hat
        _CACHE["c5_512"] = dict(sel=sel, B=S / (float(N) ** 3 * n_t), A=A, g=g, grad=grad.astype(np.float32))
    return _CACHE["c5_512"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_bispec_512(gpu, precision, tol):
    """Every count (stored table, pair-sum rule) and a wave-complete triplet sample against the oracle."""
    w = fieldgen.WORKLOADS["bispec_512_lognormal"]
    fields = _fields_cached("bispec_512_lognormal")
    tuples, counts = _golden_64shell_counts()
    ref = _c5_sample_reference()
    plan, B, bins, quot = _gpu_run(fields, 3, w["n_shells"], w["width"], precision)
    assert _integral(quot)
    assert np.array_equal(plan.tuples, tuples) and np.array_equal(plan.counts, counts)
    _pair_sum_check(plan.tuples, plan.counts, w["N"], w["n_shells"], w["width"])
    waves = {(int(t[1]) - 1) % 8 for t in tuples[ref["sel"]]}
    assert waves == set(range(8))
    got = B[0, ref["sel"]]
    rel = _rel(got, ref["B"])
    scaled = float(np.max(np.abs(got - ref["B"]) / ref["A"]))
    record_error("512^3 bispectrum, 64 unit shells (lognormal): sample", PRECISION_NAMES[precision],
                 n_tuples=len(got), rel_l2=rel, max_scaled=scaled)
    assert rel < tol
    assert scaled < tol
    plan.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,bwd_precision", [(0, 0), (2, 2), (2, 1)])
def test_bispec_512_gradient(gpu, precision, bwd_precision):
    """The benchmark's backward at 512^3 against the FP64 oracle gradient, for a loss that
    weights only the sample's triplets (so the oracle needs only the sample's fields); the
    last case is the benchmark's pairing, an FP16-split forward and a BF16-split adjoint."""
    import torch
    import paper_1904_11055_amd as ps
    fields = _fields_cached("bispec_512_lognormal")
    ref = _c5_sample_reference()
    plan = ps.Plan(512, 3, 64, 1.0, precision=precision, device="cuda:0")
    x = torch.from_numpy(fields).to("cuda:0").requires_grad_(True)
    B = ps.polyspectrum(x, plan)
    plan.precision = bwd_precision           # the adjoint's arithmetic
    B.backward(torch.from_numpy(ref["g"])[None].to("cuda:0"))
    grad = x.grad[0].cpu().numpy()
    del x, B
    grel = _rel(grad, ref["grad"])
    label = PRECISION_NAMES[precision] if bwd_precision == precision else \
        f"{PRECISION_NAMES[precision]} fwd / {PRECISION_NAMES[bwd_precision]} bwd"
    record_error("512^3 bispectrum, 64 unit shells (lognormal): gradient of a sample-supported loss",
                 label, grad_rel_l2=grel)
    assert grel < 1e-4
    plan.close()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------------------
# 256^3 trispectrum, 24 shells of width 2
# ---------------------------------------------------------------------------------------
@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_trispec_256_lognormal(gpu, precision, tol):
    """A sample of every shell block (counts via integer pair counts, B and the scaled error)."""
    w = fieldgen.WORKLOADS["trispec_256_lognormal"]
    N, nb, width = w["N"], w["n_shells"], w["width"]
    fields = _fields_cached("trispec_256_lognormal")
    plan, B, bins, quot = _gpu_run(fields, 4, nb, width, precision)
    assert _integral(quot)
    shells = [1, 2, 3, 8, 12, 17, 23, 24]
    sample = _sample(plan.tuples, shells)
    key = ("c3", tuple(shells))
    if key not in _CACHE:
        say(f"oracle on {len(sample)} sampled quadrilaterals")
        d = O.shell_fields(fields[0].astype(np.float64), nb, width, shells)
        n_t = O.polygon_counts_exact(N, 4, nb, width, sample)
        S = _subset_sums(d, shells, sample)
        A = _subset_sums(d, shells, sample, absolute=True) / (float(N) ** 3 * n_t)
        _CACHE[key] = (n_t, S / (float(N) ** 3 * n_t), A)
    n_ref, B_ref, A = _CACHE[key]
    idx = {tuple(int(v) for v in t): n for n, t in enumerate(plan.tuples)}
    sel = [idx[t] for t in sample]
    assert np.array_equal(plan.counts[sel], n_ref)
    rel = _rel(B[0, sel], B_ref)
    scaled = float(np.max(np.abs(B[0, sel] - B_ref) / A))
    record_error("256^3 trispectrum, 24 shells of width 2 (lognormal): sample", PRECISION_NAMES[precision],
                 n_tuples=len(sel), rel_l2=rel, max_scaled=scaled)
    assert rel < tol
    assert scaled < tol
    plan.close()


def _recursion_check(plan, N, order, nb, width):
    """sum_s n(t, s) = prod_j |S_{t_j}| - n(t) for (n-1)-tuples t whose vector sums always land in a shell.

    n(t) comes from an order n-1 plan on the same grid; the identity holds at any size.
    """
    import paper_1904_11055_amd as ps
    lower = ps.Plan(N, order - 1, nb, width, device="cuda:0")
    n_low = {tuple(int(v) for v in t): int(c) for t, c in zip(lower.tuples, lower.counts)}
    lower.close()
    table = {tuple(int(v) for v in t): int(c) for t, c in zip(plan.tuples, plan.counts)}
    S = O.shell_mode_counts(N, nb, width)
    checked = 0
    for h in itertools.combinations_with_replacement(range(1, nb + 1), order - 1):
        if 2 * sum(h) + len(h) > 2 * nb + 1:
            continue
        tot = sum(table.get(tuple(sorted(h + (s,))), 0) for s in range(1, nb + 1))
        assert tot == int(np.prod([S[u - 1] for u in h])) - n_low.get(h, 0), h
        checked += 1
    assert checked > 0


# Orders 5 and 6: the sampled tuples are gated on the raw sums (relative L2) and on each
# tuple's error relative to its term magnitude sum_x |prod d|, because a tuple with few
# polygons is a small residual of cancelling products.  The rounding of the float32 shell
# fields enters each of the n factors, so the gates stated for n = 3 are scaled by n / 3.
# The errors of B itself are measured and reported too.
@pytest.mark.parametrize("name,shells", [("quadspec_256_lognormal", [1, 2, 8, 15, 16]),
                                         ("pentaspec_256_lognormal", [1, 2, 5, 7, 8])])
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_high_order_256_lognormal(gpu, name, shells, precision, tol):
    import torch
    import paper_1904_11055_amd as ps
    w = fieldgen.WORKLOADS[name]
    N, order, nb, width = w["N"], w["order"], w["n_shells"], w["width"]
    fields = _fields_cached(name)
    plan = ps.Plan(N, order, nb, width, precision=precision, device="cuda:0")
    plan.shells(torch.from_numpy(fields).to("cuda:0"))
    B, S = (a.cpu().numpy()[0] for a in plan.contract(raw=True))
    _, quot = plan.candidates()
    assert _integral(quot)
    _recursion_check(plan, N, order, nb, width)
    sample = _sample(plan.tuples, shells)
    key = (name, tuple(shells))
    if key not in _CACHE:
        say(f"oracle on {len(sample)} sampled tuples of order {order}")
        dhat = O.polyspec.rfftn(fields[0].astype(np.float64))
        d = O.shell_fields_from_hat(dhat, N, nb, width, shells)
        by_shell = {s: d[n] for n, s in enumerate(shells)}
        _CACHE[key] = (O.polygon_counts_exact(N, order, nb, width, sample),
                       O.tuple_product_sums(by_shell, sample),
                       O.tuple_product_sums({s: np.abs(v) for s, v in by_shell.items()}, sample))
    n_ref, S_ref, A_ref = _CACHE[key]
    idx = {tuple(int(v) for v in t): n for n, t in enumerate(plan.tuples)}
    sel = [idx[t] for t in sample]
    assert np.array_equal(plan.counts[sel], n_ref)
    rel = _rel(S[sel], S_ref)
    scaled = float(np.max(np.abs(S[sel] - S_ref) / A_ref))
    B_ref = S_ref / (float(N) ** 3 * n_ref)
    record_error(f"256^3 order {order}, {nb} unit shells (lognormal): sample", PRECISION_NAMES[precision],
                 n_tuples=len(sel), sums_rel_l2=rel, max_scaled=scaled, B_rel_l2=_rel(B[sel], B_ref),
                 B_max_rel=float(np.max(np.abs(B[sel] - B_ref) / np.abs(B_ref))),
                 B_median_rel=float(np.median(np.abs(B[sel] - B_ref) / np.abs(B_ref))))
    assert rel < tol * order / 3
    assert scaled < tol * order / 3
    plan.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (2, 1e-4)])
def test_bispec_1024_streamed_interpolation(gpu, precision, tol):
    """1024^3 in streamed mode, forward and backward; the resident path cannot hold this size
    (its shell fields alone take 275 GB).

    delta_512 is the 512^3 benchmark field restricted to the modes of the shells' box, and
    delta_1024 its band-limited interpolation (every 512^3 mode times 8 on a 1024^3 grid).
    The modes are the same, so the counts are equal; d_s^1024 at even points is 8 d_s^512
    and no product of three fields has a mode beyond 3 K_e < 256, so B_1024 = 8^3 B_512.
    For L = sum_t g_t B_t, L_1024(I delta) = 512 L_512(delta); the adjoint of the
    interpolation I takes a band-limited field b to 8 b at the even points, so the
    1024^3 gradient at even points is 64 times the 512^3 gradient.  The 512^3 side is itself
    checked against the oracle above (test_bispec_512, test_bispec_512_gradient).
    """
    import torch
    import paper_1904_11055_amd as ps
    w = fieldgen.WORKLOADS["bispec_1024_streamed"]
    nb, width, K = w["n_shells"], w["width"], 64
    say("generating the 512^3 lognormal field and its band-limited versions on 512^3 and 1024^3")
    field = _fields_cached(w["spectrum_of"])[0]

    def real_field(n):
        hs = torch.from_numpy(fieldgen.zero_padded_half_spectrum(field, n, K)).to("cuda:0")
        x = torch.fft.irfftn(hs, s=(n, n, n)).to(torch.float32)[None].contiguous()
        del hs
        torch.cuda.empty_cache()
        return x

    rng = np.random.default_rng(7)
    p512 = ps.Plan(512, 3, nb, width, precision=precision, device="cuda:0")
    g = torch.from_numpy(rng.standard_normal((1, p512.n_closing))).to("cuda:0")
    x = real_field(512)
    p512.shells(x)
    B512 = p512.contract().cpu().numpy()
    grad512 = p512.backward(g).cpu().numpy()
    counts512 = p512.counts.copy()
    p512.close()
    del x
    torch.cuda.empty_cache()
    say("1024^3 streamed plan")
    x = real_field(1024)
    p1024 = ps.Plan(1024, 3, nb, width, precision=precision, flags=ps.STREAM_SLABS, device="cuda:0")
    assert p1024.slab_planes < 1024
    assert np.array_equal(p1024.counts, counts512)
    _, quot = p1024.candidates()
    assert _integral(quot)
    p1024.shells(x)
    B1024 = p1024.contract().cpu().numpy()
    grad1024 = p1024.backward(g)[:, ::2, ::2, ::2].cpu().numpy()
    rel_b = np.linalg.norm(B1024 - 512.0 * B512) / np.linalg.norm(512.0 * B512)
    rel_g = np.linalg.norm(grad1024 - 64.0 * grad512) / np.linalg.norm(64.0 * grad512)
    say(f"streamed 1024^3 ({1024 // p1024.slab_planes} slabs) vs resident 512^3: B {rel_b:.2e}, gradient {rel_g:.2e}")
    assert rel_b < tol
    assert rel_g < 1e-4
    p1024.close()
    del x
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------------------
# 128^3 x 8 differentiable bispectrum, 24 unit shells
# ---------------------------------------------------------------------------------------
def _c4_reference():
    if "c4" not in _CACHE:
        w = fieldgen.WORKLOADS["bispec_grad_128x8"]
        N, nb, width = w["N"], w["n_shells"], w["width"]
        fields = fieldgen.workload_fields("bispec_grad_128x8")
        target_field = fieldgen.gaussian_field(N, w["target_seed"]).astype(np.float32).astype(np.float64)
        T = O.polyspectrum(target_field, 3, nb, width)["B"]
        refs = []
        for b in range(len(fields)):
            say(f"oracle forward + gradient for field {b}")
            ref = O.polyspectrum(fields[b].astype(np.float64), 3, nb, width, return_fields=True)
            grad = O.gradient(fields[b].astype(np.float64), 3, nb, width, 2.0 * (ref["B"] - T), result=ref)
            refs.append(dict(B=ref["B"], counts=ref["counts"], grad=grad, tuples=ref["tuples"],
                             fields=ref["fields"] if b == 0 else None))
        _CACHE["c4"] = (fields, T, refs)
    return _CACHE["c4"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (2, 1e-4)])
def test_bispec_grad_128x8(gpu, precision, tol):
    """Batch of 8 Gaussian fields, loss sum_t (B_t - T_t)^2 with T from a ninth field: every
    field's B and gradient against the FP64 oracle; in FP32 also FP64 central differences."""
    import torch
    import paper_1904_11055_amd as ps
    w = fieldgen.WORKLOADS["bispec_grad_128x8"]
    N, nb, width = w["N"], w["n_shells"], w["width"]
    fields, T, refs = _c4_reference()
    plan = ps.Plan(N, 3, nb, width, batch=8, precision=precision, device="cuda:0")
    x = torch.from_numpy(fields).to("cuda:0").requires_grad_(True)
    B = ps.polyspectrum(x, plan)
    Tt = torch.from_numpy(T).to("cuda:0")[None]
    loss = ((B - Tt) ** 2).sum()
    loss.backward()
    g = x.grad.cpu().numpy()
    Bh = B.detach().cpu().numpy()
    rels, grels = [], []
    for b, ref in enumerate(refs):
        assert np.array_equal(plan.counts, ref["counts"])
        rels.append(_rel(Bh[b], ref["B"]))
        grels.append(_rel(g[b], ref["grad"]))
    record_error("128^3 x 8 bispectrum, 24 unit shells (Gaussian k^-2), loss sum (B - T)^2",
                 PRECISION_NAMES[precision], rel_l2_worst_field=max(rels), grad_rel_l2_worst_field=max(grels))
    assert max(rels) < tol
    assert max(grels) < 1e-4
    if precision == 0:
        _central_differences_check(fields[0].astype(np.float64), refs[0], T, nb, width, g[0])
    plan.close()


def _central_differences_check(delta, ref, T, nb, width, g_gpu, n_voxels=64, eps=1e-3):
    """dL/d delta at random voxels by FP64 central differences of L = sum_t (B_t - T_t)^2.

    Moving delta[y] by e adds e c_s(x - y) to every shell field (c_s the unit-shell
    field, the same inverse transform of the mask), so each difference needs the shifted
    unit fields and the product sums S_t(+e), S_t(-e), not new transforms.  Both sums are
    accumulated in one pass over x0-planes, with no grid-sized temporaries.
    """
    N = delta.shape[0]
    t, n_t = ref["tuples"], ref["counts"]
    d = ref["fields"]
    c = O.count_fields(N, nb, width)
    norm = float(N) ** 3 * n_t
    pairs = O.pair_list(nb)
    pi, pj = pairs[:, 0] - 1, pairs[:, 1] - 1
    row = {(int(a), int(b)): n for n, (a, b) in enumerate(pairs)}
    rows = np.array([row[(int(a), int(b))] for a, b in t[:, :2]])
    cols = t[:, 2] - 1
    step = 8192   # points per block: the pair products stay a few MB

    def sums_pm(y):
        acc = np.zeros((2, len(pairs), nb))
        for i0 in range(N):
            cs = np.roll(c[:, (i0 - y[0]) % N], shift=(int(y[1]), int(y[2])), axis=(1, 2)).reshape(nb, -1)
            blk = d[:, i0].reshape(nb, -1)
            for x0 in range(0, N * N, step):
                for k, sgn in enumerate((1.0, -1.0)):
                    f = blk[:, x0:x0 + step] + (sgn * eps) * cs[:, x0:x0 + step]
                    acc[k] += (f[pi] * f[pj]) @ f.T
        return acc[0][rows, cols], acc[1][rows, cols]

    rng = np.random.default_rng(64)
    ys = rng.integers(0, N, size=(n_voxels, 3))
    fd = np.empty(n_voxels)
    say(f"central differences at {n_voxels} voxels (FP64 oracle sums)")
    for i, y in enumerate(ys):
        sp, sm = sums_pm(y)
        fd[i] = (np.sum((sp / norm - T) ** 2) - np.sum((sm / norm - T) ** 2)) / (2 * eps)
    got = g_gpu[ys[:, 0], ys[:, 1], ys[:, 2]]
    rel = np.linalg.norm(got - fd) / np.linalg.norm(fd)
    say(f"GPU gradient vs central differences at {n_voxels} voxels: relative L2 {rel:.2e}")
    record_error("128^3 x 8 bispectrum: GPU gradient vs FP64 central differences (64 voxels)", "fp32",
                 fd_rel_l2=rel)
    assert rel < 1e-4


@pytest.mark.parametrize("precision", [0, 2])
def test_trispec_grad_128_lognormal(gpu, precision):
    """Order-4 gradient at 128^3 (12 shells of width 2) against the FP64 oracle."""
    import torch
    import paper_1904_11055_amd as ps
    N, nb, width = 128, 12, 2.0
    delta = fieldgen.lognormal_field(N, 61).astype(np.float32)
    key = ("tri128",)
    if key not in _CACHE:
        say("oracle forward + order-4 gradient at 128^3")
        ref = O.polyspectrum(delta.astype(np.float64), 4, nb, width, return_fields=True)
        gref = O.gradient(delta.astype(np.float64), 4, nb, width, 2.0 * ref["B"], result=ref)
        _CACHE[key] = (ref["B"], ref["counts"], gref)
    B_ref, counts, gref = _CACHE[key]
    plan = ps.Plan(N, 4, nb, width, precision=precision, device="cuda:0")
    x = torch.from_numpy(delta)[None].to("cuda:0").requires_grad_(True)
    B = ps.polyspectrum(x, plan)
    loss = (B ** 2).sum()
    loss.backward()
    g = x.grad.cpu().numpy()[0]
    assert np.array_equal(plan.counts, counts)
    Bh = B.detach().cpu().numpy()[0]
    tol = 1e-5 if precision == 0 else 1e-4
    rel, grel = _rel(Bh, B_ref), _rel(g, gref)
    record_error("128^3 trispectrum, 12 shells of width 2 (lognormal), loss sum B^2", PRECISION_NAMES[precision],
                 rel_l2=rel, grad_rel_l2=grel)
    assert rel < tol
    assert grel < 1e-4
    plan.close()
