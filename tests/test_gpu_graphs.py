"""CG iterations replayed as HIP graphs (options.graphs = 1) against the
same iterations launched kernel by kernel (graphs = 0, the default): the
results and reports must be bit-identical, on both precision paths, across
repeated solves on one operator (graph reuse), after new scalings and with a
different number of right-hand sides (recapture)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1803_08333_amd as rf
    assert torch.cuda.is_available()
    return torch, rf


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_is_bit_identical(precision):
    torch, rf = _gpu()
    m = rf.Mesh(*synth.torus(24, 12))
    start = torch.from_numpy(synth.complex_start(m.N, 11)).cuda()
    ops = [rf.Operator(m, 0.7, power_start=start, precision=precision, graphs=g) for g in (1, 0)]
    kh, pol = synth.plane_waves(3, 6)
    e = ops[0].rhs_planewave(kh, pol)
    runs = []
    for op in ops:
        out = []
        for rhs in (e, e, e[:1]):                       # replay, replay, new nrhs
            j, st, info = op.solve(rhs, tol=1e-9, maxit=400)
            out.append((j, st, [(i["iters"], i["restarts"], i["rel_residual"]) for i in info]))
        a, b, g, _ = op.scalings()
        op.set_scalings(1.3 * a, 0.8 * b, g)            # new scalars: recapture
        j, st, info = op.solve(e, tol=1e-9, maxit=400)
        out.append((j, st, [(i["iters"], i["restarts"], i["rel_residual"]) for i in info]))
        runs.append(out)
    for (ja, sa, ia), (jb, sb, ib) in zip(*runs):
        assert sa == sb == 0
        assert ia == ib
        assert torch.equal(ja, jb)
    assert max(it for it, _, _ in runs[0][0][2]) > 4      # long enough to replay both graphs
