"""The allocation-free batched weight solve against the allocating one.

mgm_batched_weights_noalloc runs the same kernel as mgm_batched_weights, with
the singular-system flag in the library's per-GPU device array instead of a
buffer allocated per call, so its weights must equal the other entry point's
bit for bit. Two calls in a row, the second on a smaller batch, check that
nothing of the first call's state leaks into the second; a singular batch
followed by a regular one checks that the flag the first raised is cleared.
"""
import numpy as np
import pytest

import synth
from paper_2204_06154_amd import mgm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _inputs(wl, k):
    sten = mgm.stencils(wl.xyz, k)
    return (torch.tensor(wl.xyz, device="cuda"), torch.tensor(wl.normals, device="cuda"),
            torch.tensor(sten, device="cuda"))


@pytest.mark.parametrize("phs,deg,k", [(1, 3, 50), (2, 2, 30)])
def test_noalloc_weights_equal_the_allocating_entry_point(phs, deg, k):
    big = synth.star_workload(6001, n_probe=20000)
    small = synth.torus_workload(1003)
    for wl in (big, small):  # the second call has the smaller batch
        print(f"[no-alloc] N={len(wl.xyz)} k={k} phs={phs} deg={deg}", flush=True)
        d_x, d_n, d_s = _inputs(wl, k)
        ref = mgm.batched_weights(d_x, d_n, d_s, phs, deg).cpu().numpy()
        out = torch.full((len(wl.xyz), k), float("nan"), dtype=torch.float64, device="cuda")
        mgm.batched_weights(d_x, d_n, d_s, phs, deg, d_weights=out, noalloc=True)
        got = out.cpu().numpy()
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_noalloc_flag_is_cleared_between_calls():
    t = np.linspace(0, 2 * np.pi, 300, endpoint=False)
    x = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], axis=1)  # collinear stencils: singular systems
    sten = mgm.stencils(x, 20)
    d_x = torch.tensor(x, device="cuda")
    d_s = torch.tensor(sten, device="cuda")
    out = torch.empty((300, 20), dtype=torch.float64, device="cuda")
    print("[no-alloc] singular batch", flush=True)
    with pytest.raises(mgm.MgmError) as ei:
        mgm.batched_weights(d_x, d_x, d_s, 1, 2, d_weights=out, noalloc=True)
    assert ei.value.status == -4
    wl = synth.sphere_workload(2000)
    d_x, d_n, d_s = _inputs(wl, 30)
    print("[no-alloc] regular batch after the singular one", flush=True)
    out = torch.empty((2000, 30), dtype=torch.float64, device="cuda")
    mgm.batched_weights(d_x, d_n, d_s, 1, 2, d_weights=out, noalloc=True)
    ref = mgm.batched_weights(d_x, d_n, d_s, 1, 2).cpu().numpy()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), ref.view(np.uint64))
