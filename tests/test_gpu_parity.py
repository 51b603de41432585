"""GPU parity of the HIP path against the FP64 oracle (small and medium grids).

Tolerances: polygon counts bit-exact; B within 1e-5 relative (L2 over the closing
tuples) for the FP32 contraction and 1e-4 for the split-precision contractions;
gradients within 1e-4 relative (L2 over the grid).
"""
import os

import numpy as np
import pytest

import fieldgen
import oracle as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
_CACHE = {}


def _ps():
    import paper_1904_11055_amd as ps
    return ps


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _run(delta, order, nb, width, precision=0, flags=0, box_length=0.0):
    import torch
    ps = _ps()
    delta = np.asarray(delta, dtype=np.float32)
    if delta.ndim == 3:
        delta = delta[None]
    plan = ps.Plan(delta.shape[-1], order, nb, width, batch=delta.shape[0], precision=precision,
                   flags=flags, box_length=box_length, device="cuda:0")
    x = torch.from_numpy(delta).to("cuda:0")
    plan.shells(x)
    B, S = plan.contract(raw=True)
    torch.cuda.synchronize()
    return plan, B.cpu().numpy(), S.cpu().numpy()


@pytest.fixture(scope="module")
def bispec64():
    delta = fieldgen.workload_fields("bispec_64")[0]
    ref = O.polyspectrum(delta.astype(np.float64), 3, 16, 1.0, return_fields=True)
    return delta, ref


def test_counts_bit_exact_64(gpu, bispec64):
    delta, ref = bispec64
    plan, B, _ = _run(delta, 3, 16, 1.0)
    assert np.array_equal(plan.tuples, ref["tuples"])
    assert np.array_equal(plan.counts, ref["counts"])
    gold = np.loadtxt(os.path.join(GOLDEN, "bispec_64_counts.txt"), dtype=np.int64)
    assert np.array_equal(plan.counts, gold[:, 3])
    bins, quot = plan.candidates()
    assert np.abs(quot - np.rint(quot)).max() < 1e-6
    plan.close()


def test_shell_fields_64(gpu, bispec64):
    delta, ref = bispec64
    plan, _, _ = _run(delta, 3, 16, 1.0)
    f = plan.fields().cpu().numpy()[0]
    d = ref["fields"]
    scale = np.abs(d).max(axis=(1, 2, 3))
    err = np.abs(f - d).max(axis=(1, 2, 3)) / scale
    assert err.max() < 2e-6, err
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_bispectrum_64(gpu, bispec64, precision, tol):
    delta, ref = bispec64
    plan, B, S = _run(delta, 3, 16, 1.0, precision=precision)
    assert _rel(B[0], ref["B"]) < tol
    assert _rel(S[0], ref["sums"]) < tol
    plan.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_bispectrum_ragged_shells(gpu, precision):
    # 20 shells: two shell blocks, the second ragged; 240 pairs over 15 pair blocks
    delta = fieldgen.lognormal_field(64, 9).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 3, 20, 1.0)
    plan, B, _ = _run(delta, 3, 20, 1.0, precision=precision)
    assert np.array_equal(plan.counts, ref["counts"])
    assert _rel(B[0], ref["B"]) < (1e-5 if precision == 0 else 1e-4)
    plan.close()


# Degenerate configurations: one shell, an empty shell, a field with no power in any
# shell (the FP16 scaling then meets all-zero fields), and a resident plan on the
# largest grid.
@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (2, 1e-4)])
def test_single_shell(gpu, order, precision, tol):
    delta = fieldgen.lognormal_field(32, 70 + order).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), order, 1, 1.0)
    plan, B, _ = _run(delta, order, 1, 1.0, precision=precision)
    assert np.array_equal(plan.tuples, ref["tuples"]) and len(ref["tuples"]) == 1
    assert np.array_equal(plan.counts, ref["counts"])
    assert _rel(B[0], ref["B"]) < tol
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (2, 1e-4)])
def test_empty_shell(gpu, precision, tol):
    """Width 1/2: shell 1, (1/4 <= |q| < 3/4), holds no mode, so no tuple with it closes."""
    assert O.shell_mode_counts(32, 6, 0.5)[0] == 0
    delta = fieldgen.gaussian_field(32, 73).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 3, 6, 0.5)
    plan, B, _ = _run(delta, 3, 6, 0.5, precision=precision)
    assert np.array_equal(plan.tuples, ref["tuples"])
    assert np.array_equal(plan.counts, ref["counts"])
    assert not np.any(plan.tuples == 1)              # shell 1 is in no closing tuple
    bins, quot = plan.candidates()
    assert np.any(bins == 1) and np.all(quot[np.any(bins == 1, axis=1)] == 0.0)
    assert _rel(B[0], ref["B"]) < tol
    plan.close()


@pytest.mark.parametrize("order", [3, 5])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_field_without_shell_power(gpu, order, precision):
    """A constant field has power only at q = 0, which no shell holds: every B is exactly 0."""
    ps = _ps()
    delta = np.full((32, 32, 32), 0.75, dtype=np.float32)
    plan, B, S = _run(delta, order, 4, 1.0, precision=precision, flags=ps.NAN_GUARD)
    assert np.all(np.isfinite(B)) and np.all(np.abs(S) < 1e-6 * 0.75 ** order * 32 ** (3 * order))
    _, Bz, _ = _run(np.zeros((32, 32, 32), dtype=np.float32), order, 4, 1.0, precision=precision,
                    flags=ps.NAN_GUARD)
    assert np.array_equal(Bz, np.zeros_like(Bz))
    plan.close()


def test_largest_grid_resident(gpu):
    """N = 1024 without streaming (4 shells): the band-limited interpolation of a 256^3 field
    gives B_1024 = (4^3)^3 B_256 with the same counts."""
    import torch
    ps = _ps()
    field = fieldgen.lognormal_field(256, 74)
    res = {}
    for n in (256, 1024):
        hs = torch.from_numpy(fieldgen.zero_padded_half_spectrum(field, n, 4)[None]).to("cuda:0")
        plan = ps.Plan(n, 3, 4, 1.0, flags=ps.INPUT_HALF_SPECTRUM, device="cuda:0")
        assert plan.slab_planes == n
        plan.shells(hs)
        res[n] = (plan.counts.copy(), plan.contract().cpu().numpy())
        plan.close()
        del hs
        torch.cuda.empty_cache()
    assert np.array_equal(res[1024][0], res[256][0])
    assert _rel(res[1024][1], 64.0 ** 3 * res[256][1]) < 1e-5


def test_unit_spectrum_gives_one(gpu):
    plan, B, _ = _run(fieldgen.unit_spectrum_field(32), 3, 10, 1.0)
    np.testing.assert_allclose(B[0], 1.0, rtol=1e-5)   # the FP32 gate
    plan.close()


def test_power_spectrum(gpu):
    delta = fieldgen.gaussian_field(32, 4).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 2, 14, 1.0)
    plan, B, _ = _run(delta, 2, 14, 1.0)
    assert np.array_equal(plan.counts, ref["counts"])
    np.testing.assert_allclose(B[0], ref["B"], rtol=1e-5)
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_trispectrum(gpu, precision, tol):
    delta = fieldgen.lognormal_field(32, 6).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 4, 7, 1.0)
    plan, B, _ = _run(delta, 4, 7, 1.0, precision=precision)
    assert np.array_equal(plan.tuples, ref["tuples"])
    assert np.array_equal(plan.counts, ref["counts"])
    assert _rel(B[0], ref["B"]) < tol
    plan.close()


# Orders 5 and 6 (Sec. 4.2 runs the estimator for pentagons and hexagons): pair x
# triple and triple x triple tiles, alias-free at 64^3 and aliased at 32^3.
#
# At these orders a tuple with few polygons has a sum S_t that is a small residual
# of large cancelling products (sum_x |prod d| / |S_t| reaches 6e4 here), so any
# float32 evaluation misses such B_t by that factor times the rounding unit, and a
# relative L2 over B is dominated by them.  The gates are therefore the relative L2
# over the raw sums and the error of every tuple relative to its term magnitude
# A_t = sum_x |prod_j d_{t_j}[x]|, each scaled by n / 3 from the gates stated for
# n = 3, since the rounding of the float32 shell fields enters each of the n factors.
_HIGH = {}


def _high_ref(N, order, nb, aliased):
    key = (N, order, nb)
    if key not in _HIGH:
        delta = fieldgen.lognormal_field(N, 30 + order).astype(np.float32)
        ref = O.polyspectrum(delta.astype(np.float64), order, nb, 1.0, allow_aliasing=aliased, return_fields=True)
        ref["magnitude"] = O.product_sums(np.abs(ref.pop("fields")), ref["tuples"])
        _HIGH[key] = (delta, ref)
    return _HIGH[key]


@pytest.mark.parametrize("N,order,nb,aliased", [(64, 5, 12, False), (32, 5, 6, True), (64, 6, 8, False),
                                                (32, 6, 5, True)])
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_orders_five_and_six(gpu, N, order, nb, aliased, precision, tol):
    ps = _ps()
    delta, ref = _high_ref(N, order, nb, aliased)
    plan, B, S = _run(delta, order, nb, 1.0, precision=precision, flags=ps.ALLOW_ALIASING if aliased else 0)
    assert np.array_equal(plan.tuples, ref["tuples"])
    assert np.array_equal(plan.counts, ref["counts"])
    assert _rel(S[0], ref["sums"]) < tol * order / 3
    assert np.max(np.abs(S[0] - ref["sums"]) / ref["magnitude"]) < tol * order / 3
    np.testing.assert_allclose(B[0], S[0] / (float(N) ** 3 * ref["counts"]), rtol=1e-14)
    plan.close()


@pytest.mark.parametrize("order,nb", [(5, 4), (6, 3)])
def test_unit_spectrum_gives_one_high_orders(gpu, order, nb):
    plan, B, _ = _run(fieldgen.unit_spectrum_field(32), order, nb, 1.0)
    np.testing.assert_allclose(B[0], 1.0, rtol=1e-5)
    plan.close()


# Streamed plans: the last two inverse passes and the contraction run one x1-slab at
# a time (8 slabs of 8 planes at 64^3, 8 slabs of the smallest 4-plane slab at 32^3).
@pytest.mark.parametrize("order,nb,precision,tol", [(3, 16, 0, 1e-5), (3, 16, 1, 1e-4), (3, 16, 2, 1e-4),
                                                    (4, 9, 2, 1e-4), (2, 20, 0, 1e-5)])
def test_streamed_matches_oracle_and_resident(gpu, bispec64, order, nb, precision, tol):
    import torch
    ps = _ps()
    delta = bispec64[0] if order == 3 else fieldgen.lognormal_field(64, 40 + order).astype(np.float32)
    ref = bispec64[1] if order == 3 else O.polyspectrum(delta.astype(np.float64), order, nb, 1.0)
    plan = ps.Plan(64, order, nb, 1.0, precision=precision, flags=ps.STREAM_SLABS, slab_planes=8,
                   device="cuda:0")
    assert plan.slab_planes == 8
    x = torch.from_numpy(delta[None]).to("cuda:0")
    plan.shells(x)
    B1 = plan.contract().cpu().numpy()
    B2 = plan.contract().cpu().numpy()
    assert np.array_equal(B1, B2)                       # fixed slab order: bitwise reruns
    assert np.array_equal(plan.counts, ref["counts"])
    assert _rel(B1[0], ref["B"]) < tol
    _, Bres, _ = _run(delta, order, nb, 1.0, precision=precision)
    assert _rel(B1[0], Bres[0]) < tol
    plan.close()


@pytest.mark.parametrize("order,precision,tol", [(3, 2, 1e-4), (5, 0, 1e-5 * 5 / 3)])
def test_streamed_batch_and_smallest_slab(gpu, order, precision, tol):
    import torch
    ps = _ps()
    nb = 10 if order == 3 else 4
    fields = np.stack([fieldgen.lognormal_field(32, s).astype(np.float32) for s in (50, 51)])
    plan = ps.Plan(32, order, nb, 1.0, batch=2, precision=precision, flags=ps.STREAM_SLABS, slab_planes=4,
                   device="cuda:0")
    plan.shells(torch.from_numpy(fields).to("cuda:0"))
    B, S = (a.cpu().numpy() for a in plan.contract(raw=True))
    for b in range(2):
        ref = O.polyspectrum(fields[b].astype(np.float64), order, nb, 1.0)
        assert np.array_equal(plan.counts, ref["counts"])
        assert _rel(S[b], ref["sums"]) < tol
    plan.close()


@pytest.mark.parametrize("order,N,nb,batch,planes,precision,tol", [
    (3, 32, 8, 1, 4, 0, 1e-4), (3, 32, 8, 1, 8, 1, 1e-4), (3, 64, 12, 2, 8, 1, 1e-4), (4, 32, 7, 1, 4, 2, 1e-4)])
def test_streamed_backward(gpu, order, N, nb, batch, planes, precision, tol):
    """The adjoint slab by slab: against the FP64 oracle gradient and the resident plan's gradient."""
    import torch
    ps = _ps()
    fields = np.stack([fieldgen.lognormal_field(N, 60 + b).astype(np.float32) for b in range(batch)])
    rng = np.random.default_rng(order)
    grads = {}
    for flags, kw in ((ps.STREAM_SLABS, dict(slab_planes=planes)), (0, {})):
        plan = ps.Plan(N, order, nb, 1.0, batch=batch, precision=precision, flags=flags, device="cuda:0", **kw)
        g = rng.standard_normal((batch, plan.n_closing)) if not grads else grads["g"]
        plan.shells(torch.from_numpy(fields).to("cuda:0"))
        plan.contract()
        grads["g"] = g
        grads[flags] = plan.backward(torch.from_numpy(g).to("cuda:0")).cpu().numpy()
        plan.close()
    streamed, resident = grads[ps.STREAM_SLABS], grads[0]
    # the same adjoint arithmetic on both sides agrees to float32 rounding; in FP16 mode a
    # streamed plan runs the BF16 adjoint (its field scales are per slab) and the resident
    # one the FP16 adjoint, so there the two agree to the split tolerance
    assert _rel(streamed, resident) < (1e-6 if precision != ps.SPLIT_FP16 else tol)
    for b in range(batch):
        d64 = fields[b].astype(np.float64)
        ref = O.polyspectrum(d64, order, nb, 1.0, return_fields=True)
        gref = O.gradient(d64, order, nb, 1.0, grads["g"][b], result=ref)
        assert _rel(streamed[b], gref) < tol
        assert _rel(resident[b], gref) < tol


def test_streamed_plan_limits(gpu):
    import torch
    ps = _ps()
    plan = ps.Plan(32, 3, 6, 1.0, flags=ps.STREAM_SLABS, device="cuda:0")
    assert plan.slab_planes == 32                          # 6 shells at 32^3 fit one 2 GiB slab
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_set_slab_planes(plan.handle, 2)       # below the smallest slab at N = 32
    assert e.value.status == 1
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_set_slab_planes(plan.handle, 12)      # not a power of two
    assert e.value.status == 1
    ps.polyspec_set_slab_planes(plan.handle, 16)
    assert ps.polyspec_slab_planes(plan.handle) == 16
    plan.shells(torch.from_numpy(fieldgen.gaussian_field(32, 3).astype(np.float32)[None]).to("cuda:0"))
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_set_slab_planes(plan.handle, 8)       # workspace already sized
    assert e.value.status == 6
    with pytest.raises(ps.PolyspecError) as e:
        plan.fields()
    assert e.value.status == 6
    plan.close()
    resident = ps.Plan(32, 3, 6, 1.0, device="cuda:0")
    assert resident.slab_planes == 32
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_set_slab_planes(resident.handle, 8)
    assert e.value.status == 6
    resident.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (2, 1e-4)])
def test_aliased_configuration(gpu, precision, tol):
    ps = _ps()
    delta = fieldgen.gaussian_field(32, 12).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 3, 12, 1.0, allow_aliasing=True)
    plan, B, _ = _run(delta, 3, 12, 1.0, precision=precision, flags=ps.ALLOW_ALIASING)
    assert np.array_equal(plan.tuples, ref["tuples"])
    assert np.array_equal(plan.counts, ref["counts"])
    assert _rel(B[0], ref["B"]) < tol
    plan.close()


def test_width_two_shells(gpu):
    delta = fieldgen.lognormal_field(64, 2).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 3, 9, 2.0)
    plan, B, _ = _run(delta, 3, 9, 2.0)
    assert np.array_equal(plan.counts, ref["counts"])
    assert _rel(B[0], ref["B"]) < 1e-5
    plan.close()


def test_half_spectrum_input_and_box_length(gpu):
    import torch
    ps = _ps()
    delta = fieldgen.gaussian_field(32, 14).astype(np.float32)
    L = 1000.0
    ref = O.polyspectrum(delta.astype(np.float64), 3, 8, 1.0, box_length=L)
    hs = np.fft.rfftn(delta.astype(np.float64)).astype(np.complex64)
    plan = ps.Plan(32, 3, 8, 1.0, flags=ps.INPUT_HALF_SPECTRUM, box_length=L, device="cuda:0")
    plan.shells(torch.from_numpy(hs)[None].to("cuda:0"))
    B = plan.contract().cpu().numpy()[0]
    assert _rel(B, ref["B"]) < 1e-5
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (2, 1e-4)])
def test_batch_matches_single(gpu, precision, tol):
    fields = np.stack([fieldgen.gaussian_field(32, s) for s in (21, 22, 23)]).astype(np.float32)
    plan, B, _ = _run(fields, 3, 8, 1.0, precision=precision)
    for b in range(3):
        ref = O.polyspectrum(fields[b].astype(np.float64), 3, 8, 1.0)
        assert _rel(B[b], ref["B"]) < tol
    plan.close()


def test_reruns_are_bitwise_equal(gpu):
    import torch
    delta = fieldgen.gaussian_field(64, 3).astype(np.float32)
    plan, B1, _ = _run(delta, 3, 16, 1.0, precision=1)
    B2 = plan.contract().cpu().numpy()
    plan.shells(torch.from_numpy(delta)[None].to("cuda:0"))
    B3 = plan.contract().cpu().numpy()
    assert np.array_equal(B1, B2) and np.array_equal(B1, B3)
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 1e-4), (2, 1e-4)])
def test_gradient_matches_oracle(gpu, precision, tol):
    import torch
    ps = _ps()
    N, nb = 32, 8
    delta = fieldgen.gaussian_field(N, 31).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 3, nb, 1.0, return_fields=True)
    rng = np.random.default_rng(0)
    g = rng.standard_normal(len(ref["B"]))
    gref = O.gradient(delta.astype(np.float64), 3, nb, 1.0, g, result=ref)
    plan = ps.Plan(N, 3, nb, 1.0, precision=precision, device="cuda:0")
    x = torch.from_numpy(delta)[None].to("cuda:0").requires_grad_(True)
    B = ps.polyspectrum(x, plan)
    B.backward(torch.from_numpy(g)[None].to("cuda:0"))
    assert _rel(x.grad.cpu().numpy()[0], gref) < tol
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 1e-4), (2, 1e-4)])
@pytest.mark.parametrize("N,nb,width,flags", [(32, 7, 1.0, 0), (32, 9, 1.0, 2), (64, 6, 2.0, 0)])
def test_trispectrum_gradient_matches_oracle(gpu, precision, tol, N, nb, width, flags):
    """Order-4 adjoint (incl. an aliased plan and width 2) against the FP64 oracle gradient."""
    import torch
    ps = _ps()
    allow = bool(flags & ps.ALLOW_ALIASING)
    delta = fieldgen.lognormal_field(N, 51).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 4, nb, width, return_fields=True, allow_aliasing=allow)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(len(ref["B"]))
    gref = O.gradient(delta.astype(np.float64), 4, nb, width, g, result=ref, allow_aliasing=allow)
    plan = ps.Plan(N, 4, nb, width, precision=precision, flags=flags, device="cuda:0")
    x = torch.from_numpy(delta)[None].to("cuda:0").requires_grad_(True)
    B = ps.polyspectrum(x, plan)
    assert np.array_equal(plan.counts, ref["counts"])
    B.backward(torch.from_numpy(g)[None].to("cuda:0"))
    assert _rel(x.grad.cpu().numpy()[0], gref) < tol
    plan.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 1e-4), (2, 1e-4)])
def test_trispectrum_gradient_more_than_32_shells(gpu, precision, tol):
    """34 shells of width 1/4 at 64^3 (alias-free: 4 x 34.5 / 4 <= 64; the thinnest shells
    hold no mode): the order-4 adjoint with four 16-shell chunks of u and two 32-row blocks
    of m (a ragged last block of each), against the FP64 oracle gradient, and the forward."""
    import torch
    ps = _ps()
    N, nb, width = 64, 34, 0.25
    key = ("tri_grad_34",)
    if key not in _CACHE:
        delta = fieldgen.lognormal_field(N, 52).astype(np.float32)
        ref = O.polyspectrum(delta.astype(np.float64), 4, nb, width, return_fields=True)
        g = np.random.default_rng(2).standard_normal(len(ref["B"]))
        gref = O.gradient(delta.astype(np.float64), 4, nb, width, g, result=ref)
        _CACHE[key] = (delta, ref["counts"], ref["B"], g, gref)
    delta, counts, Bref, g, gref = _CACHE[key]
    plan = ps.Plan(N, 4, nb, width, precision=precision, device="cuda:0")
    x = torch.from_numpy(delta)[None].to("cuda:0").requires_grad_(True)
    B = ps.polyspectrum(x, plan)
    assert np.array_equal(plan.counts, counts)
    # the forward too: 38 pair blocks, more than one workgroup's LDS holds as shared
    # operands, so the tiles run in groups that each form their own blocks
    assert _rel(B.detach().cpu().numpy()[0], Bref) < (1e-5 if precision == 0 else 1e-4)
    if precision == 2:   # the plan keeps its FP16 tile groups when switched to FP32
        plan.precision = ps.FP32
        assert _rel(plan.contract().cpu().numpy()[0], Bref) < 1e-5
        plan.precision = ps.SPLIT_FP16
    B.backward(torch.from_numpy(g)[None].to("cuda:0"))
    err = _rel(x.grad.cpu().numpy()[0], gref)
    from conftest import PRECISION_NAMES, record_error
    record_error("64^3 trispectrum, 34 shells of width 1/4 (lognormal): gradient of sum g_t B_t",
                 PRECISION_NAMES[precision], grad_rel_l2=err)
    assert err < tol
    plan.close()


@pytest.mark.timeout(600)
def test_trispectrum_gradient_more_than_32_shells_streamed(gpu):
    """The 34-shell order-4 plan above run slab by slab (8 slabs of 8 planes, FP32): the
    64-shell adjoint form writing its fields for the slab's own transforms, against the
    FP64 oracle gradient and the resident plan."""
    import torch
    ps = _ps()
    N, nb, width = 64, 34, 0.25
    key = ("tri_grad_34",)
    if key not in _CACHE:
        delta = fieldgen.lognormal_field(N, 52).astype(np.float32)
        ref = O.polyspectrum(delta.astype(np.float64), 4, nb, width, return_fields=True)
        g = np.random.default_rng(2).standard_normal(len(ref["B"]))
        gref = O.gradient(delta.astype(np.float64), 4, nb, width, g, result=ref)
        _CACHE[key] = (delta, ref["counts"], ref["B"], g, gref)
    delta, counts, Bref, g, gref = _CACHE[key]
    x = torch.from_numpy(delta)[None].to("cuda:0")
    out = {}
    for flags, kw in ((ps.STREAM_SLABS, dict(slab_planes=8)), (0, {})):
        plan = ps.Plan(N, 4, nb, width, flags=flags, device="cuda:0", **kw)
        plan.shells(x)
        B = plan.contract().cpu().numpy()[0]
        assert np.array_equal(plan.counts, counts)
        assert _rel(B, Bref) < 1e-5
        out[flags] = plan.backward(torch.from_numpy(g)[None].to("cuda:0")).cpu().numpy()[0]
        plan.close()
    assert _rel(out[ps.STREAM_SLABS], gref) < 1e-4
    assert _rel(out[ps.STREAM_SLABS], out[0]) < 1e-6


def test_trispectrum_backward_limits(gpu):
    """More than 64 shells: the order-4 backward reports UNSUPPORTED (the plan is refused
    before any field is needed)."""
    import torch
    ps = _ps()
    plan = ps.Plan(128, 4, 65, 0.5, flags=ps.ALLOW_ALIASING, device="cuda:0")
    with pytest.raises(ps.PolyspecError) as e:
        plan.backward(torch.ones(1, plan.n_closing, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == 7
    plan.close()


def test_state_and_guard_errors(gpu):
    import torch
    ps = _ps()
    plan = ps.Plan(32, 3, 8, 1.0, flags=ps.NAN_GUARD, device="cuda:0")
    with pytest.raises(ps.PolyspecError) as e:
        plan.contract()
    assert e.value.status == 6
    with pytest.raises(ps.PolyspecError) as e:
        plan.backward(torch.zeros(1, plan.n_closing, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == 6
    bad = torch.zeros(1, 32, 32, 32, device="cuda:0")
    bad[0, 1, 2, 3] = float("nan")
    plan.shells(bad)
    with pytest.raises(ps.PolyspecError) as e:
        plan.contract()
    assert e.value.status == 4
    plan.close()


def test_precision_switch_after_shells(gpu):
    import torch
    ps = _ps()
    delta = fieldgen.lognormal_field(64, 17).astype(np.float32)
    ref = O.polyspectrum(delta.astype(np.float64), 3, 16, 1.0)
    plan = ps.Plan(64, 3, 16, 1.0, precision=ps.SPLIT_BF16, device="cuda:0")
    plan.shells(torch.from_numpy(delta)[None].to("cuda:0"))
    for prec, tol in ((ps.SPLIT_FP16, 1e-4), (ps.FP32, 1e-5), (ps.SPLIT_BF16, 1e-4)):
        plan.precision = prec
        B = plan.contract().cpu().numpy()[0]
        assert _rel(B, ref["B"]) < tol, prec
    plan.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_issued_flops_cover_the_algorithmic_work(gpu, precision):
    """Every launched tile counts, so the issued work is at least 2 flops per tuple and point."""
    ps = _ps()
    plan = ps.Plan(64, 3, 16, 1.0, precision=precision, device="cuda:0")
    G = 64 ** 3
    terms = 1 if precision == 0 else 3
    ctr = ps.polyspec_issued_flops(plan.handle, "contract")
    adj = ps.polyspec_issued_flops(plan.handle, "adj_gemm")
    assert ctr >= 2.0 * plan.n_closing * G * terms
    assert adj >= 2.0 * plan.n_closing * G * terms
    assert ps.polyspec_issued_flops(plan.handle, "shell_p3") == 0.0
    plan.close()


def _scaled_error(B, ref, tol_name=""):
    """max_t |B_t - B_ref,t| / A_t with A_t = sum_x |prod_j d_{t_j}[x]| / (N^3 n_t): the error
    relative to the size of the terms summed, meaningful where B_t itself is near 0."""
    d = ref["fields"]
    N = d.shape[-1]
    A = O.product_sums(np.abs(d), ref["tuples"]) / (float(N) ** 3 * ref["counts"])
    return float(np.max(np.abs(np.asarray(B) - ref["B"]) / A))


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
@pytest.mark.parametrize("order,nb", [(3, 16), (4, 9)])
def test_per_tuple_scaled_error(gpu, bispec64, order, nb, precision, tol):
    """Every tuple, not only the norm: the error of each B_t relative to its term magnitude."""
    delta = bispec64[0]
    ref = O.polyspectrum(delta.astype(np.float64), order, nb, 1.0, return_fields=True)
    plan, B, _ = _run(delta, order, nb, 1.0, precision=precision)
    assert np.array_equal(plan.counts, ref["counts"])
    err = _scaled_error(B[0], ref)
    from conftest import PRECISION_NAMES, record_error
    record_error(f"64^3 order {order}, {nb} shells (Gaussian k^-2)", PRECISION_NAMES[precision],
                 rel_l2=_rel(B[0], ref["B"]), max_scaled=err)
    assert err < tol
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (2, 1e-4)])
@pytest.mark.parametrize("order,nb", [(3, 8), (4, 6)])
def test_half_spectrum_backward(gpu, order, nb, precision, tol):
    """Half-spectrum input: the gradient comes back as dL/dRe X + i dL/dIm X on the half spectrum."""
    import torch
    ps = _ps()
    N = 32
    delta = fieldgen.lognormal_field(N, 81).astype(np.float32)
    X = np.fft.rfftn(delta.astype(np.float64)).astype(np.complex64)
    X64 = X.astype(np.complex128)
    ref = O.polyspectrum_from_hat(X64, N, order, nb, 1.0, return_fields=True)
    rng = np.random.default_rng(order)
    g = rng.standard_normal(len(ref["B"]))
    Gref = O.gradient_half_spectrum(N, order, nb, 1.0, ref["tuples"], ref["counts"], ref["fields"], g)
    plan = ps.Plan(N, order, nb, 1.0, precision=precision, flags=ps.INPUT_HALF_SPECTRUM, device="cuda:0")
    x = torch.from_numpy(X)[None].to("cuda:0").requires_grad_(True)
    B = ps.polyspectrum(x, plan)
    assert np.array_equal(plan.counts, ref["counts"])
    B.backward(torch.from_numpy(g)[None].to("cuda:0"))
    G = x.grad.cpu().numpy()[0]
    assert G.dtype == np.complex64
    assert np.all(G[O.shell_id_grid(N, nb, 1.0) == 0] == 0)       # modes in no shell get nothing
    assert _rel(G, Gref) < tol
    plan.close()


def test_autograd_refuses_stale_fields(gpu):
    """Two forwards on one plan, then the backward of the first: its fields are gone, so it raises."""
    import torch
    ps = _ps()
    plan = ps.Plan(32, 3, 8, 1.0, device="cuda:0")
    x1 = torch.from_numpy(fieldgen.gaussian_field(32, 1).astype(np.float32))[None].to("cuda:0").requires_grad_(True)
    x2 = torch.from_numpy(fieldgen.gaussian_field(32, 2).astype(np.float32))[None].to("cuda:0").requires_grad_(True)
    B1 = ps.polyspectrum(x1, plan)
    B2 = ps.polyspectrum(x2, plan)
    with pytest.raises(RuntimeError, match="another forward"):
        B1.sum().backward()
    B2.sum().backward()                  # the latest forward still differentiates
    assert torch.isfinite(x2.grad).all() and x1.grad is None
    with pytest.raises(ValueError):
        plan.backward(torch.ones(1, plan.n_closing + 1, dtype=torch.float64, device="cuda:0"))
    plan.close()


def test_caller_workspace(gpu):
    """polyspec_set_workspace with caller memory: results equal the Plan's; misuse is refused."""
    import ctypes
    import torch
    ps = _ps()
    delta = fieldgen.gaussian_field(32, 5).astype(np.float32)
    ref_plan, Bref, _ = _run(delta, 3, 8, 1.0)
    assert ref_plan._workspace is not None           # the binding hands torch memory to the library
    ref_plan.close()
    h = ps.polyspec_plan(32, 3, 8, 1.0, stream=ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    need = ps.polyspec_workspace_size(h)
    buf = torch.empty(need + 512, dtype=torch.uint8, device="cuda:0")
    base = buf.data_ptr() + (-buf.data_ptr()) % 256
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_set_workspace(h, base, need - 1)          # too small
    assert e.value.status == 1
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_set_workspace(h, base + 8, need)          # not 256-byte aligned
    assert e.value.status == 1
    ps.polyspec_set_workspace(h, base, need)
    with pytest.raises(ps.PolyspecError) as e:
        ps.polyspec_set_workspace(h, base, need)              # already set
    assert e.value.status == 6
    x = torch.from_numpy(delta)[None].to("cuda:0")
    out = torch.empty(1, len(Bref[0]), dtype=torch.float64, device="cuda:0")
    ps.polyspec_shells(h, x.data_ptr())
    ps.polyspec_contract(h, out.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), Bref)
    ps.polyspec_destroy(h)
    del buf


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-4), (2, 1e-4)])
def test_more_than_64_shells(gpu, precision, tol):
    """80 shells of width 1/2 at 128^3 (alias-free: 3 x 40.25 <= 128): the tile contraction
    with eight staged shell blocks, every closing triplet against the oracle (counts
    bit-exact, B and the per-tuple error relative to the term magnitude)."""
    N, nb, width = 128, 80, 0.5
    key = ("more_than_64",)
    if key not in _CACHE:
        delta = fieldgen.lognormal_field(N, 93).astype(np.float32)
        ref = O.polyspectrum(delta.astype(np.float64), 3, nb, width, return_fields=True)
        ref["A"] = O.product_sums(np.abs(ref["fields"]), ref["tuples"]) / (float(N) ** 3 * ref["counts"])
        del ref["fields"]
        _CACHE[key] = (delta, ref)
    delta, ref = _CACHE[key]
    plan, B, _ = _run(delta, 3, nb, width, precision=precision)
    assert plan.n_closing == len(ref["B"]) > 25424 // 2
    assert np.array_equal(plan.tuples, ref["tuples"])
    assert np.array_equal(plan.counts, ref["counts"])
    scaled = float(np.max(np.abs(B[0] - ref["B"]) / ref["A"]))
    from conftest import PRECISION_NAMES, record_error
    record_error("128^3 bispectrum, 80 shells of width 1/2 (lognormal)", PRECISION_NAMES[precision],
                 n_tuples=len(ref["B"]), rel_l2=_rel(B[0], ref["B"]), max_scaled=scaled)
    assert _rel(B[0], ref["B"]) < tol
    assert scaled < tol
    ps = _ps()
    import torch
    with pytest.raises(ps.PolyspecError) as e:    # the adjoint holds at most 64 shells
        plan.backward(torch.zeros(1, plan.n_closing, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == 7
    plan.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (2, 1e-4)])
def test_more_than_64_shells_streamed(gpu, precision, tol):
    """The 80-shell plan above run slab by slab (16 slabs of 8 planes): every closing triplet
    against the oracle, and against the resident plan."""
    import torch
    ps = _ps()
    N, nb, width = 128, 80, 0.5
    key = ("more_than_64",)
    if key not in _CACHE:
        delta = fieldgen.lognormal_field(N, 93).astype(np.float32)
        ref = O.polyspectrum(delta.astype(np.float64), 3, nb, width, return_fields=True)
        ref["A"] = O.product_sums(np.abs(ref["fields"]), ref["tuples"]) / (float(N) ** 3 * ref["counts"])
        del ref["fields"]
        _CACHE[key] = (delta, ref)
    delta, ref = _CACHE[key]
    x = torch.from_numpy(delta)[None].to("cuda:0")
    plan = ps.Plan(N, 3, nb, width, precision=precision, flags=ps.STREAM_SLABS, slab_planes=8, device="cuda:0")
    assert plan.slab_planes == 8
    plan.shells(x)
    B = plan.contract().cpu().numpy()
    assert np.array_equal(plan.counts, ref["counts"])
    from conftest import PRECISION_NAMES, record_error
    scaled = float(np.max(np.abs(B[0] - ref["B"]) / ref["A"]))
    record_error("128^3 bispectrum, 80 shells of width 1/2, streamed (16 slabs)", PRECISION_NAMES[precision],
                 n_tuples=len(ref["B"]), rel_l2=_rel(B[0], ref["B"]), max_scaled=scaled)
    assert _rel(B[0], ref["B"]) < tol
    assert scaled < tol
    plan.close()
    _, Br, _ = _run(delta, 3, nb, width, precision=precision)
    assert _rel(B[0], Br[0]) < tol

