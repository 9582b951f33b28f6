"""tnqe_subspace_noalloc (the entry point for callers that cannot allocate)
against tnqe_subspace with a caller workspace, through the C ABI (MI355X)."""
import os

import numpy as np
import pytest

import paper_2404_10223_amd as T
import tnqe_synth as synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _close(a, b, tol=1e-10):
    H, S, E = a[:3]
    Hr, Sr, Er = b[:3]
    assert np.abs(H - Hr).max() <= tol * np.abs(Hr).max()
    assert np.abs(S - Sr).max() <= tol
    assert abs(E - Er) <= tol * (1 + abs(Er))


def test_noalloc_matches_workspace_entry():
    import torch
    ctx = T.Context(0)
    try:
        cap = T.lib().tnqe_noalloc_capacity()
        assert cap == 256 << 20
        big, small = synth.make_config(2), synth.make_config(1)
        assert ctx.workspace_size(small, chi=small.chi) < ctx.workspace_size(big, chi=big.chi) <= cap
        # two calls in a row, the second with a smaller input; each against
        # the workspace entry point on the same inputs and the stored oracle
        for prob in (big, small):
            print(f"noalloc N={prob.N} chi={prob.chi} M={prob.M}", flush=True)
            free0 = torch.cuda.mem_get_info()[0]
            got = ctx.subspace_noalloc(prob, chi=prob.chi)
            free1 = torch.cuda.mem_get_info()[0]
            ws = torch.empty(ctx.workspace_size(prob, chi=prob.chi), dtype=torch.uint8, device="cuda")
            ref = ctx.subspace(prob, chi=prob.chi, workspace=ws)
            _close(got, ref)
            g = np.load(os.path.join(GOLD, f"oracle_{prob.name}.npz"))
            _close(got, (g["H"], g["S"], float(g["E"])))
            assert 0 < got[4]["ws_peak_bytes"] <= cap
            if prob is small:
                assert free1 == free0, (free0, free1)   # the second call allocated no device memory
        # inputs whose bound exceeds the scratch are refused before any work
        c3 = synth.make_config(3)
        assert ctx.workspace_size(c3, chi=c3.chi) > cap
        with pytest.raises(T.TnqeError) as e:
            ctx.subspace_noalloc(c3, chi=c3.chi)
        assert e.value.status == -6
        again = ctx.subspace_noalloc(small, chi=small.chi)
        _close(again, got)
    finally:
        ctx.close()
