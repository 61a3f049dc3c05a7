"""GPU parity of every kernel variant of the SelInv level sweep.

The level schedule (Section 2.1: block J runs once every block holding a row
of R_J is done) launches one kernel per level, in a variant chosen by the
level's width and its blocks' sizes (asi_sweep_plan reports which). These
cases make every variant run and compare the whole result on S, entry by
entry, with the oracle: a seeded layered factor built so that its levels
fall in every width band (including levels of more than 3,072 blocks with and
without heavy blocks, and more than 1,024 blocks of |R_J| > 128, with 2x2
pivots in each), and a 7-point diffusion grid at 40^3 whose real levels reach
the wavefront-per-block variant.
"""
import numpy as np
import pytest

from oracle import core as oc
from workloads import diffusion3d_7pt, ildl_bk, nested_multicolor_grid
from workloads.layered import layered_factor

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4
ALL_VARIANTS = ["small", "split", "group128", "group256", "group512", "big256", "big1024"]


def _factor(name):
    if name == "layered":
        return layered_factor(seed=1)
    if name == "diff40_tau1e-3":
        return ildl_bk(diffusion3d_7pt(40, 1.0, 3), nested_multicolor_grid((40, 40, 40)), 1e-3)
    raise KeyError(name)


EXPECTED = {"layered": ALL_VARIANTS, "diff40_tau1e-3": ["small", "group128", "group256", "group512"]}


@pytest.fixture(scope="module")
def oracle_results():
    cache = {}

    def get(name):
        if name not in cache:
            F = _factor(name)
            S = oc.pattern(F)
            Zo = oc.selinv(F, S)
            No = oc.ninv(F, S, 3, 0.1)
            cache[name] = (F, S, Zo, No)
        return cache[name]
    return get


@pytest.mark.parametrize("name", ["layered", "diff40_tau1e-3"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_level_variant_matches_the_oracle(oracle_results, name, precision):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    print(f"[level variants] case={name} precision={precision}", flush=True)
    F, S, Zo, No = oracle_results(name)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    plan = s.sweep_plan()
    print(f"  n={F.n} |S|={S.nnz} 2x2={int((F.piv == 1).sum())} plan={plan}", flush=True)
    for v in EXPECTED[name]:
        assert plan[v] > 0, f"variant {v} not launched"
    s.set_sweep("levels")
    Lv, dd, ds = upload_factors(F)
    # per-call factor pointers, then the loaded factor with NInv beside it
    Z1 = s.selinv(Lv, dd, ds, precision=precision)
    s.load_factor(Lv, dd, ds)
    Z2, N2 = s.selinv_ninv(p=3, delta=0.1, precision=precision)
    s.sync()
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for tag, Z in (("per-call", Z1), ("loaded", Z2)):
        e = oc.entry_error(S, Z.cpu().numpy(), Zo)
        print(f"  SelInv {tag}: e max={e.max():.2e} p99={np.quantile(e, 0.99):.2e}", flush=True)
        assert e.max() <= tol
    en = oc.entry_error(S, N2.cpu().numpy(), No).max()
    print(f"  NInv beside the sweep: e max={en:.2e}", flush=True)
    assert en <= tol
    # the launches themselves, counted by the library's tracing
    s.profile(True)
    s.selinv(precision=precision)
    prof = s.profile_read()
    s.profile(False)
    s.sync()
    nlaunch = prof["selinv"][0] + prof["selinv_big"][0]
    assert nlaunch == sum(plan.values())
