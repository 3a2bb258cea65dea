"""Helpers shared by the GPU parity tests: device transfer and the comparison
rules (projection within 1e-5 * ||x|| * max|weight|; codes equal except at
oracle near-edge components, which are counted; keys equal for every table
whose K codes are all outside the near-edge band)."""
import numpy as np
import pytest
import torch


def dev():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        t = torch.from_numpy(a.view(np.int64))
    elif a.dtype == np.uint32:
        t = torch.from_numpy(a.view(np.int32))
    elif a.dtype == np.uint16:
        t = torch.from_numpy(a.view(np.int16))
    else:
        t = torch.from_numpy(a)
    t = t.to(dev())
    return t if dtype is None else t.to(dtype)


def to_host(t, dtype=None):
    a = t.detach().cpu().numpy()
    return a if dtype is None else a.view(dtype)


def compare_hash(out, ref, x64, K, L, weight_max=1.0, exact=False, what=""):
    """Check GPU outputs against the oracle's.  Returns the near-edge count."""
    n, m = ref["codes"].shape
    if out.get("proj") is not None:
        yg = to_host(out["proj"]).astype(np.float64)
        tol = 1e-5 * np.linalg.norm(x64, axis=1) * weight_max
        err = np.abs(yg - ref["y"]).max(axis=1) if n else np.zeros(0)
        bad = np.nonzero(err > tol)[0]
        assert bad.size == 0, f"{what}: projection off at rows {bad[:5]} err {err[bad[:5]]} tol {tol[bad[:5]]}"
    near = ref["near"]
    if out.get("codes") is not None:
        cg = to_host(out["codes"])
        diff = cg != ref["codes"]
        if exact:
            assert not diff.any(), f"{what}: {diff.sum()} codes differ (exact mode)"
        else:
            outside = diff & ~near
            assert not outside.any(), (f"{what}: {outside.sum()} codes differ outside the "
                                       f"near-edge band, first at {np.argwhere(outside)[:3]}")
    if out.get("keys") is not None:
        kg = to_host(out["keys"], np.uint64)
        tab_near = near.reshape(n, L, K).any(axis=2).T  # [L][n]
        diff = kg != ref["keys"]
        if exact:
            assert not diff.any(), f"{what}: {diff.sum()} keys differ (exact mode)"
        else:
            outside = diff & ~tab_near
            assert not outside.any(), f"{what}: {outside.sum()} keys differ outside the band"
    return int(near.sum())
