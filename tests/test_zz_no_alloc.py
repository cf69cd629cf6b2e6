"""mcx_detpost_device_noalloc, the detected-photon post-processing entry point
for callers that cannot allocate device memory, against mcx_detpost_device
(which allocates its workspace) on the same records, through the C ABI.

Both run the same kernels: each workgroup sums its records into an FP64
histogram with LDS atomics (in no fixed order) and the partial sums are
added in workgroup order, so the two agree to FP64 rounding order (1e-12
relative), record counts and re-weighted weights exactly.  Two calls in a
row, the second smaller, check that the shared workspace keeps nothing from
the first call that matters."""
import sys

import numpy as np
import pytest

import oracle
from paper_1711_03244_amd import mcx

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def records(seed, nrec, ndet, npath, t_hi):
    """Synthetic detector records {det, nscat, w, t, L_1..L_npath}."""
    rng = np.random.default_rng(seed)
    rec = np.empty((nrec, 4 + npath), np.float32)
    rec[:, 0] = rng.integers(0, ndet, nrec)
    rec[:, 1] = rng.integers(0, 500, nrec)
    rec[:, 2] = rng.uniform(1e-4, 1.0, nrec)
    rec[:, 3] = rng.uniform(0.0, t_hi, nrec)
    rec[:, 4:] = rng.uniform(0.0, 50.0, (nrec, npath))
    return rec


def run_both(rec, spec, dmua):
    import torch
    drec = torch.as_tensor(rec).cuda()
    dd = torch.as_tensor(np.asarray(dmua, np.float32)).cuda() if dmua is not None else None
    res = []
    for noalloc in (False, True):
        out = torch.full((spec["ndet"], 2 + spec["ngates"]), float("nan"), dtype=torch.float64,
                         device="cuda")
        w = torch.full((len(rec),), float("nan"), dtype=torch.float64, device="cuda")
        mcx.mcx_detpost_device(drec, spec, dd, out=out, weight=w, noalloc=noalloc)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), w.cpu().numpy()))
    return res


def check_oracle(out, w, rec, spec, dmua):
    ref, wref = oracle.detected_postprocess(rec, spec["nphoton"], spec["ndet"], spec["t0"],
                                            spec["dt"], spec["ngates"], dmua)
    assert np.array_equal(out[:, 0], ref[:, 0])
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-15 * np.abs(ref[:, 1:]).max())
    assert np.allclose(w, wref, rtol=1e-14, atol=0)


def test_noalloc_equals_allocating_call_twice_second_smaller():
    cases = [
        (dict(ndet=4, npath=2, t0=0.0, dt=0.1, ngates=50, nphoton=10**6), 30000, (0.002, -0.001)),
        (dict(ndet=3, npath=2, t0=0.5, dt=0.25, ngates=10, nphoton=10**5), 5000, None),
    ]
    for i, (spec, nrec, dmua) in enumerate(cases):
        say(f"[gpu] no-alloc post-processing call {i}: nrec={nrec} spec={spec} dmua={dmua}")
        rec = records(10 + i, nrec, spec["ndet"], spec["npath"], spec["t0"] + 6.0)
        (a, wa), (b, wb) = run_both(rec, spec, dmua)
        assert np.array_equal(a[:, 0], b[:, 0])
        assert np.allclose(b, a, rtol=1e-12, atol=1e-15 * np.abs(a[:, 1:]).max())
        assert np.array_equal(wa, wb)
        check_oracle(b, wb, rec, spec, dmua)


def test_noalloc_many_records_several_passes():
    # 300 detectors x 52 columns need two histogram passes; 2e5 records use
    # 782 workgroups in the allocating call and 128 in the no-alloc one
    spec = dict(ndet=300, npath=3, t0=0.0, dt=0.1, ngates=50, nphoton=10**7)
    dmua = (0.001, 0.0, -0.0005)
    for i, nrec in enumerate((200_000, 40_000)):
        say(f"[gpu] no-alloc post-processing, {nrec} records, two passes")
        rec = records(20 + i, nrec, spec["ndet"], spec["npath"], 6.0)
        (a, wa), (b, wb) = run_both(rec, spec, dmua)
        assert np.array_equal(a[:, 0], b[:, 0])
        assert np.allclose(b, a, rtol=1e-12, atol=1e-15 * np.abs(a[:, 1:]).max())
        assert np.array_equal(wa, wb)
        check_oracle(b, wb, rec, spec, dmua)


def test_noalloc_empty_input():
    import torch
    spec = dict(ndet=2, npath=1, t0=0.0, dt=1.0, ngates=3, nphoton=100)
    out = torch.full((2, 5), float("nan"), dtype=torch.float64, device="cuda")
    mcx.mcx_detpost_device(torch.zeros((0, 5), device="cuda"), spec, out=out, noalloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.zeros((2, 5)))
