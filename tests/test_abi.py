"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side classification (no GPU work) agrees with the oracle's
independent classification.  No compute call needs a device here."""
import os
import re

import numpy as np
import pytest

import workloads as W
from conftest import ROOT
from oracle import classify

pk = pytest.importorskip("paper_2001_07289_amd")


def _declared():
    src = open(os.path.join(ROOT, "include", "bddcso.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bddcso_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = pk.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pk.EXPORTED) == names


@pytest.mark.parametrize("make", [
    W.fig1_problem, W.config1,
    lambda: W.config2_like(n=24, H=12, L=4),
    lambda: W.config2_like(n=24, H=12, L=2),
    lambda: W.table1_problem(4),
    lambda: W.config3(n=48, nrhs=1, count=4),
], ids=["fig1", "cfg1", "3d_L4", "3d_L2", "table1_k4", "uneven"])
def test_classification_matches_oracle(make):
    p = make()
    prob = pk.Problem.from_workload(p)
    c = classify.classify(p.n_el, p.elem_sub, p.elem_subsub)
    for mask in (7, 1, 2, 4, 6):
        info = prob.info(mask)
        sel = [o for o in range(len(c.obj_nodes)) if c.obj_type[o] & mask]
        t = c.obj_type[sel]
        assert info["n_coarse"] == len(sel)
        assert info["counts"] == {"v": int(np.sum(t == 1)), "e": int(np.sum(t == 2)),
                                  "f": int(np.sum(t == 4))}
    info = prob.info()
    assert info["n_free"] == p.n_free
    assert info["n_gamma"] == int(c.is_gamma.sum())
    assert info["n_sub"] == c.n_sub


def test_rejects_non_box_subdomain():
    p = W.config1_like(n=8, H=4, L=2)
    es = p.elem_sub.copy()
    ess = p.elem_subsub.copy()
    es[0] = 3  # one element of the first subdomain moved to the last one
    ess[0] = ess[-1]
    with pytest.raises(pk.BDDCSOError) as e:
        pk.Problem(2, p.n_el, p.h, es, ess)
    assert e.value.name == "EINVAL" and "box" in str(e.value)


def test_rejects_subsubdomain_spanning_two_subdomains():
    p = W.config1_like(n=8, H=4, L=2)
    ess = p.elem_subsub.copy()
    ess[:] = 0
    with pytest.raises(pk.BDDCSOError) as e:
        pk.Problem(2, p.n_el, p.h, p.elem_sub, ess)
    assert e.value.name == "EINVAL"


def test_rejects_bad_dims():
    with pytest.raises(pk.BDDCSOError):
        pk.Problem(4, (4, 4), (0.25, 0.25), np.zeros(16), np.zeros(16))
    with pytest.raises(ValueError):
        pk.Problem(2, (4, 4), (0.25, 0.25), np.zeros(15), np.zeros(15))


def test_default_options():
    o = pk.default_options()
    assert (o.primal_mask, o.weighting, o.precision, o.coarse_solver, o.max_nrhs) == (7, 1, 0, 0, 1)
    assert o.rtol == 1e-8 and o.maxit == 1000
