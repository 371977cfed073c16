"""The oracle's ACA ranks against the maximum ranks the paper prints for its
three kernels (Sec. 5.1 figures, eps = 1e-7, N_max = 216, tensor grids of
8,000 and 27,000 particles in [-1,1]^3).

The paper does not state its ACA variant (pivot rules, stopping norm), so a
rank can differ by a few; the band is 15 % of the printed value.  The growth
the paper reports is checked exactly: at both sizes 1/r^4 needs the largest
ranks, then cos(r)/r, then 1/r, and every kernel's maximum rank grows from
8,000 to 27,000 particles.
"""
import json
import os

import pytest

from paper_2307_16303_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_max_ranks.json")
KERNELS = {"inv_r": ("laplace", 1.0), "inv_r4": ("inv_r4", 0.0), "cos_r": ("cos_r", 1.0)}


@pytest.fixture(scope="module")
def ranks(oracle_mod):
    g = json.load(open(GOLDEN))
    out = {}
    for n in g["max_rank"]:
        k = round(int(n) ** (1.0 / 3.0))
        pts = inputs.grid_points(k)
        for name, (kern, par) in KERNELS.items():
            h = oracle_mod.HODLR3D(pts, kernel=kern, param=par, leaf_size=g["leaf_size"],
                                   tol=g["tol"], **dict(box_lo=inputs.CUBE_LO,
                                                        box_side=inputs.CUBE_SIDE))
            out[(n, name)] = int(h.far()["rank"].max())
    return g, out


def test_max_ranks_within_band_of_the_paper(ranks):
    g, out = ranks
    for n, per in g["max_rank"].items():
        for name, printed in per.items():
            got = out[(n, name)]
            print(f"[paper ranks] N={n} {name}: oracle {got}, paper {printed}")
            assert abs(got - printed) <= 0.15 * printed, (n, name, got, printed)


def test_rank_growth_by_kernel_and_size(ranks):
    g, out = ranks
    for n in g["max_rank"]:
        assert out[(n, "inv_r4")] > out[(n, "cos_r")] >= out[(n, "inv_r")]
    for name in KERNELS:
        assert out[("27000", name)] > out[("8000", name)]
