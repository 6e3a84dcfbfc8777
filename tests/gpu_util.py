"""Helpers shared by the GPU tests (input upload, oracle comparison)."""
import numpy as np

import ddsynth

NEAR_TIE = 1e-12      # oracle relative gap below which either index is accepted
DIST_RTOL = 1e-12     # relative tolerance of the reported FP64 distance


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def compare_to_oracle(idx, dist, o_idx, o_dist, o_second, data_states=None, q_states=None, C=None):
    """Indices equal wherever the oracle's best is clear of the runner-up by NEAR_TIE;
    distances within DIST_RTOL.  Returns the number of audited near ties."""
    idx = np.asarray(idx)
    dist = np.asarray(dist)
    clear = o_second > o_dist * (1.0 + NEAR_TIE)
    bad = np.flatnonzero(clear & (idx != o_idx))
    assert bad.size == 0, f"{bad.size} index mismatches, first at {bad[:5]}: gpu {idx[bad[:5]]} oracle {o_idx[bad[:5]]}"
    tie = np.flatnonzero(~clear)
    # on near ties the GPU's point must be as near as the oracle's (to rounding)
    np.testing.assert_allclose(dist, o_dist, rtol=DIST_RTOL, atol=1e-300)
    return tie.size


def assert_matches_oracle_solve(got, ref, history=True):
    """A GPU dd_solve result against the oracle's DD loop (fe.dd_solve) from the
    same initial association: iteration count, association history (when both
    recorded it) or final association, changed counts; u, strains and stresses
    to 1e-10 of their maxima (CG / direct solve rounding), distances to 1e-9."""
    assert got["iterations"] == ref.iterations
    if history:
        for i, h in enumerate(ref.history):
            assert np.array_equal(got["history"][i], h), f"association differs at iteration {i}"
    assert np.array_equal(got["idx"], ref.idx)
    assert list(got["changed"]) == ref.changed
    np.testing.assert_allclose(got["u"], ref.u, rtol=0, atol=1e-10 * np.abs(ref.u).max())
    np.testing.assert_allclose(got["eps"], ref.eps, rtol=0, atol=1e-10 * np.abs(ref.eps).max())
    np.testing.assert_allclose(got["sig"], ref.sig, rtol=0, atol=1e-10 * np.abs(ref.sig).max())
    np.testing.assert_allclose(got["d_half"], ref.d_half, rtol=1e-9)
    np.testing.assert_allclose(got["d_full"], ref.d_full, rtol=1e-9)
