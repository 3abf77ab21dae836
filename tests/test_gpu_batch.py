"""Batched V-cycles over several systems (fsi_mg_vcycle_batch): every
system's result equals its own V-cycle's bit for bit (the batched kernels run
each system's arithmetic unchanged), for systems of different mesh sizes and
level counts, sweep points and time steps, the FP64 and the mixed forms
(bf16, fp16, FP32 storage and the FP32 solid-block policy in one batch), and
more systems than one launch takes (16)."""

import sys

import numpy as np
import pytest

from gpu_common import dev, host
from synth import config, fourier_coefficients

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problems():
    from paper_1709_05660_amd import Problem
    base = config("c1_2d_128x32")
    specs = [base.with_(nx=32, ny=8, levels=2, mu_s=2.0e4, u_peak=0.1, seed=2001),
             base.with_(nx=64, ny=16, levels=3, mu_s=3.0e5, u_peak=0.25, seed=2002, transient=True),
             base.with_(nx=128, ny=32, levels=4, mu_s=5.0e5, u_peak=0.2, seed=2003),
             base.with_(nx=32, ny=8, levels=2, mu_s=8.0e5, u_peak=0.05, seed=2004, transient=True),
             base.with_(nx=64, ny=16, levels=3, mu_s=1.0e4, u_peak=0.3, seed=2005)]
    return [Problem(s, fourier_coefficients(2, s.seed)) for s in specs]


def _check(mgs, probs):
    from paper_1709_05660_amd import MG
    rng = np.random.default_rng(5)
    rs = [dev(rng.standard_normal(p.n)) for p in probs]
    single = [host(m.vcycle(r)) for m, r in zip(mgs, rs)]
    batched = [host(z) for z in MG.vcycle_batch(mgs, rs)]
    for i, (a, b) in enumerate(zip(single, batched)):
        assert np.array_equal(a, b), i
    # again: the batched launches leave nothing behind that changes a result
    again = [host(z) for z in MG.vcycle_batch(mgs, rs)]
    for a, b in zip(single, again):
        assert np.array_equal(a, b)


def test_batched_vcycle_fp64():
    from paper_1709_05660_amd import MG
    probs = _problems()
    mgs = [MG(p, precision="fp64") for p in probs]
    _check(mgs, probs)
    for m in mgs:
        m.close()


def test_batched_vcycle_mixed_forms_together():
    from paper_1709_05660_amd import MG
    probs = _problems()
    kinds = [dict(precision="bf16"), dict(precision="fp16"), dict(precision="fp32"),
             dict(precision="bf16", solid_precision="fp32"), dict(precision="bf16")]
    mgs = [MG(p, **k) for p, k in zip(probs, kinds)]
    _check(mgs, probs)
    for m in mgs:
        m.close()


def test_batched_vcycle_more_than_one_launch_takes():
    from paper_1709_05660_amd import MG, Problem
    base = config("c1_2d_128x32")
    probs = [Problem(s, fourier_coefficients(2, s.seed))
             for s in (base.with_(nx=32, ny=8, levels=2, mu_s=1.0e4 * (1 + i), seed=3000 + i,
                                  transient=bool(i % 2)) for i in range(18))]
    mgs = [MG(p, precision="bf16") for p in probs]
    _check(mgs, probs)
    for m in mgs:
        m.close()


def test_batched_vcycle_rejects_incompatible_handles():
    from paper_1709_05660_amd import MG, FsiError
    probs = _problems()[:2]
    a = MG(probs[0], precision="fp64")
    b = MG(probs[1], precision="bf16")
    r = [dev(np.ones(p.n)) for p in probs]
    with pytest.raises(FsiError):
        MG.vcycle_batch([a, b], r)
    with pytest.raises(FsiError):
        MG.vcycle_batch([a], [r[0]], [r[0]])                   # r aliased with z
    z = [dev(np.zeros(probs[0].n)) for _ in range(2)]
    with pytest.raises(FsiError):
        MG.vcycle_batch([a, a], [r[0], r[0]], z)               # one system twice
    a.close()
    b.close()
