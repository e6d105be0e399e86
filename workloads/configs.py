"""Problem descriptions for the synthetic Stokes-Darcy workloads.

A problem is a plain dict (JSON-serialisable):

  domain      [x0, x1, y0, y1]
  physics     nu_s, nu_d, alpha (BJS friction), k_bjs (the deterministic
              permeability used in the BJS term), inflow (Stokes velocity
              imposed on the whole Stokes outer boundary), p_bottom (Darcy
              pressure on y = y0; the other Darcy outer sides are no-flow)
  subdomains  list of {type: "stokes"|"darcy", rect, n: [nx, ny], region}
              Stokes subdomains first, then Darcy; each group row-major
              from the bottom-left (the numbering of Section 3.1).
  mortar      {degree: 1|2, elements: E}  discontinuous Lagrange mortar
              with E uniform elements on every interface.
  regions     list of KL regions {rect, nterm, sigma2, eta: [e1, e2],
              mean_logk}; each is an exact union of Darcy subdomains.
  rule        {kind: "tensor", m} or {kind: "sparse", level, growth}
  discretization  optional {stokes: "q2q1"|"p2p1", darcy: "trapezoidal"|"exact"}:
              the Stokes pair (Q2-Q1 on rectangles, or triangular
              Taylor-Hood P2-P1 with two triangles per rectangle) and the
              integration of the RT0 velocity mass; the default is
              Q2-Q1 with the trapezoidal mass.

Every random draw is seeded; the layouts are the coupled Stokes-over-Darcy
geometries of the paper's numerical section (Section 6), scaled to the
sizes listed for each case below.
"""
import numpy as np

PROBLEM_NAMES = ("cfg0", "cfg1", "cfg2", "cfg3")


def _grid(kind, x0, x1, y0, y1, nsx, nsy, mesh, region_of):
    out = []
    hx = (x1 - x0) / nsx
    hy = (y1 - y0) / nsy
    for jy in range(nsy):
        for jx in range(nsx):
            rect = [x0 + jx * hx, x0 + (jx + 1) * hx, y0 + jy * hy, y0 + (jy + 1) * hy]
            n = mesh(len(out), jx, jy)
            out.append({"type": kind, "rect": rect, "n": [int(n[0]), int(n[1])],
                        "region": int(region_of(jx, jy))})
    return out


def _physics():
    return {"nu_s": 1.0, "nu_d": 1.0, "alpha": 1.0, "k_bjs": 1.0,
            "inflow": [0.0, -1.0], "p_bottom": 0.0}


def _cfg0():
    stokes = _grid("stokes", 0.0, 1.0, 1.0, 2.0, 1, 1, lambda *_: (8, 8), lambda *_: -1)
    darcy = _grid("darcy", 0.0, 1.0, 0.0, 1.0, 2, 1, lambda *_: (8, 8), lambda jx, jy: jx)
    regions = [{"rect": [0.0, 0.5, 0.0, 1.0], "nterm": 2, "sigma2": 1.0, "eta": [0.2, 0.2],
                "mean_logk": 0.0},
               {"rect": [0.5, 1.0, 0.0, 1.0], "nterm": 2, "sigma2": 1.0, "eta": [0.2, 0.2],
                "mean_logk": 0.0}]
    return {"name": "cfg0", "domain": [0.0, 1.0, 0.0, 2.0], "physics": _physics(),
            "subdomains": stokes + darcy, "mortar": {"degree": 1, "elements": 2},
            "regions": regions, "rule": {"kind": "tensor", "m": 2}}


def _cfg1():
    stokes = _grid("stokes", 0.0, 1.0, 1.0, 2.0, 2, 2, lambda *_: (32, 32), lambda *_: -1)
    darcy = _grid("darcy", 0.0, 1.0, 0.0, 1.0, 4, 4, lambda *_: (32, 32),
                  lambda jx, jy: (jy // 2) * 2 + jx // 2)
    regions = []
    for ry in range(2):
        for rx in range(2):
            regions.append({"rect": [0.5 * rx, 0.5 * rx + 0.5, 0.5 * ry, 0.5 * ry + 0.5],
                            "nterm": 3, "sigma2": 1.0, "eta": [0.25, 0.1], "mean_logk": 0.0})
    return {"name": "cfg1", "domain": [0.0, 1.0, 0.0, 2.0], "physics": _physics(),
            "subdomains": stokes + darcy, "mortar": {"degree": 1, "elements": 4},
            "regions": regions, "rule": {"kind": "sparse", "level": 2, "growth": "paper"}}


def _cfg2():
    stokes = _grid("stokes", 0.0, 2.0, 1.0, 2.0, 4, 2, lambda *_: (64, 64), lambda *_: -1)
    darcy = _grid("darcy", 0.0, 2.0, 0.0, 1.0, 8, 4, lambda *_: (64, 64),
                  lambda jx, jy: (jy // 2) * 2 + jx // 4)
    regions = []
    for ry in range(2):
        for rx in range(2):
            regions.append({"rect": [1.0 * rx, 1.0 * rx + 1.0, 0.5 * ry, 0.5 * ry + 0.5],
                            "nterm": 2, "sigma2": 2.0, "eta": [0.2, 0.2], "mean_logk": 0.0})
    return {"name": "cfg2", "domain": [0.0, 2.0, 0.0, 2.0], "physics": _physics(),
            "subdomains": stokes + darcy, "mortar": {"degree": 1, "elements": 8},
            "regions": regions, "rule": {"kind": "tensor", "m": 3}}


def _cfg3(seed=3):
    rng = np.random.default_rng(seed)
    choices = np.array([16, 32, 48, 64, 96])
    sizes = []
    for _ in range(32):
        nx = int(rng.choice(choices))
        ny = int(rng.choice(choices))
        sizes.append((nx, ny))
    regions = []
    for ry in range(2):
        for rx in range(4):
            e1 = float(rng.uniform(0.05, 0.3))
            e2 = float(rng.uniform(0.05, 0.3))
            regions.append({"rect": [0.5 * rx, 0.5 * rx + 0.5, 0.5 * ry, 0.5 * ry + 0.5],
                            "nterm": 4, "sigma2": 1.0, "eta": [e1, e2], "mean_logk": 0.0})
    stokes = _grid("stokes", 0.0, 2.0, 1.0, 2.0, 4, 2, lambda *_: (64, 64), lambda *_: -1)
    darcy = _grid("darcy", 0.0, 2.0, 0.0, 1.0, 8, 4, lambda idx, jx, jy: sizes[idx],
                  lambda jx, jy: (jy // 2) * 4 + jx // 2)
    return {"name": "cfg3", "domain": [0.0, 2.0, 0.0, 2.0], "physics": _physics(),
            "subdomains": stokes + darcy, "mortar": {"degree": 2, "elements": 4},
            "regions": regions, "rule": {"kind": "sparse", "level": 3, "growth": "paper"}}


def problem(name, **overrides):
    """Return the problem dict for one named workload.

    Keyword overrides replace top-level keys or, with dotted names such as
    ``sigma2`` or ``rule``, the matching entry of every KL region / the rule.
    """
    base = {"cfg0": _cfg0, "cfg1": _cfg1, "cfg2": _cfg2, "cfg3": _cfg3}[name]()
    for key, val in overrides.items():
        if key == "sigma2":
            for r in base["regions"]:
                r["sigma2"] = float(val)
        elif key == "nterm":
            for r in base["regions"]:
                r["nterm"] = int(val)
        elif key == "mesh":
            for s in base["subdomains"]:
                s["n"] = [int(val[0]), int(val[1])]
        elif key == "darcy_mesh":
            for s in base["subdomains"]:
                if s["type"] == "darcy":
                    s["n"] = [int(val[0]), int(val[1])]
        elif key == "stokes_mesh":
            for s in base["subdomains"]:
                if s["type"] == "stokes":
                    s["n"] = [int(val[0]), int(val[1])]
        else:
            base[key] = val
    return base


def serving_stream(seed=4, duration_s=60.0, rate_hz=200.0, max_batch=256,
                   grid_sizes=None, problems=("cfg1", "cfg2", "cfg3")):
    """Poisson stream of realization batches.

    Returns a list of (arrival_time_s, problem_name, global_indices[np.int64]).
    ``grid_sizes`` maps a problem name to its number of collocation points.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        b = int(rng.integers(1, max_batch + 1))
        pname = problems[int(rng.integers(0, len(problems)))]
        n = grid_sizes[pname]
        idx = rng.integers(0, n, size=b).astype(np.int64)
        out.append((t, pname, idx))
    return out
