"""Geometry boundary (Sec. 3.2 composite panels on closed curves): curve
offsets, and panel end points checked against the node data and the curve
chain, through the C ABI on the multiply connected four-curve domain."""
import numpy as np
import pytest
import torch

from paper_1908_07392_amd import mhlp
from paper_1908_07392_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def test_curves_and_panel_ends_accepted_and_reported():
    g = wl.config5_geometry()[0]
    offs = g.curve_panel_offsets
    G = mhlp.Geometry(_t(g.node_soa()), curve_panel_offsets=offs, panel_ends=_t(g.panel_ends()))
    n, np_, got = G.info()
    assert (n, np_) == (g.n_nodes, g.n_panels)
    assert got == [int(v) for v in offs]
    # the same geometry without the optional ends gives the same operator
    G0 = mhlp.Geometry(_t(g.node_soa()), curve_panel_offsets=offs)
    P, P0 = mhlp.Plan(G, 30.0), mhlp.Plan(G0, 30.0)
    mu = _t(np.cos(3 * g.theta))
    a, b = mhlp.apply_bie(P, mu), mhlp.apply_bie(P0, mu)
    assert torch.equal(a, b)


def test_inconsistent_panel_ends_rejected():
    g = wl.config5_geometry()[0]
    offs = g.curve_panel_offsets
    ends = g.panel_ends()
    bad = ends.copy()
    bad[2, 100] += 1e-3                     # end of panel 100 moved off its node polynomial
    with pytest.raises(mhlp.MhlpError, match="panel 100 does not end where its node polynomial ends"):
        mhlp.Geometry(_t(g.node_soa()), curve_panel_offsets=offs, panel_ends=_t(bad))
    # offsets that cut the outer circle in two: its halves do not close
    wrong = [0, 256, 512, 640, 768, 896]
    with pytest.raises(mhlp.MhlpError, match="does not end where the next panel of its curve starts"):
        mhlp.Geometry(_t(g.node_soa()), curve_panel_offsets=wrong, panel_ends=_t(ends))
    with pytest.raises(mhlp.MhlpError):
        mhlp.Geometry(_t(g.node_soa()), curve_panel_offsets=[0, 500], panel_ends=_t(ends))
