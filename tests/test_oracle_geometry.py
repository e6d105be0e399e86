"""Pins of the oracle's layout and mortar maps (Section 3.1, 3.3)."""
import numpy as np
import pytest

from oracle.geometry import Layout, mortar_shape
from workloads import problem


@pytest.mark.parametrize("name,counts,M", [
    ("cfg0", (0, 2, 1), 12), ("cfg1", (4, 4, 24), 288), ("cfg2", (10, 8, 52), 1280), ("cfg3", (10, 8, 52), 960)])
def test_interface_counts_and_mortar_size(name, counts, M):
    """Interface types and mortar DOFs: E (deg + 1) per interface, twice on Gamma_ss."""
    L = Layout(problem(name))
    kinds = [f.kind for f in L.ifaces]
    assert (kinds.count("ss"), kinds.count("sd"), kinds.count("dd")) == counts
    deg = problem(name)["mortar"]["degree"]
    E = problem(name)["mortar"]["elements"]
    assert all(f.ndof == E * (deg + 1) * (2 if f.kind == "ss" else 1) for f in L.ifaces)
    assert L.M == M
    # every mortar DOF belongs to exactly two subdomains
    cnt = np.zeros(L.M, dtype=int)
    for d in L.sub_dofs:
        cnt[d] += 1
    assert np.all(cnt == 2)


def test_floating_stokes_subdomains():
    assert [i for i in range(12) if Layout(problem("cfg1")).is_floating(i)] == []
    L = Layout(problem("cfg2"))
    assert [i for i in range(L.nsub) if L.is_floating(i)] == [1, 2]


def test_mortar_shapes_partition_of_unity_and_exact_integrals():
    for deg in (1, 2):
        s = np.linspace(0, 1, 11)
        assert np.allclose(mortar_shape(deg, s).sum(axis=0), 1.0)
    L = Layout(problem("cfg3"))
    f = L.ifaces[0]
    # integral of every node shape over the whole interface equals the
    # integral over the mortar mesh, however the segment is cut
    whole = f.node_integrals(f.a, f.b)
    cuts = np.linspace(f.a, f.b, 8)
    pieces = sum(f.node_integrals(a, b) for a, b in zip(cuts[:-1], cuts[1:]))
    assert np.allclose(whole, pieces, atol=1e-15)
    # P2 shapes: endpoint nodes integrate to H/6, midpoint to 2H/3
    assert np.allclose(whole[:3], [f.H / 6, 2 * f.H / 3, f.H / 6], rtol=1e-14)
    # quadratic weight x^2 integrated exactly
    g = lambda t: t ** 2
    tot = f.node_integrals(f.a, f.b, g).sum()
    assert abs(tot - (f.b ** 3 - f.a ** 3) / 3) < 1e-15


def test_darcy_boundary_classification():
    L = Layout(problem("cfg0"))
    kinds = {}
    for be in L.darcy_boundary(1):
        kinds.setdefault(be["side"], set()).add(be["kind"])
    assert kinds == {"bottom": {"dirichlet"}, "top": {"mortar"}, "left": {"noflow"}, "right": {"mortar"}}
