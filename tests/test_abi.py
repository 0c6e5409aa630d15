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
    for mask in (7, 1, 2, 4, 6, 13, 15):
        info = prob.info(mask)
        sel = c.coarse_objects if mask == 7 else classify.classify(p.n_el, p.elem_sub, p.elem_subsub,
                                                                    primal_mask=mask).coarse_objects
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


def test_workspace_size_matches_plan_info():
    """bddcso_setup_workspace_size is host-only and equals the device bytes
    the plan reports; more right-hand sides need more workspace."""
    p = W.config1()
    prob = pk.Problem.from_workload(p)
    n1 = prob.workspace_size()
    assert n1 > 0 and n1 % 1 == 0
    assert prob.plan_stats()["device_bytes"] == n1
    assert prob.workspace_size(max_nrhs=4) > n1


def test_front_above_4gib_is_refused():
    """The front kernels address a front's entries with 32-bit byte offsets:
    one dense front of the 96^3 problem's 39,823 coarse dofs (12.7 GB) is
    refused by the planner, while its nested-dissection fronts are accepted
    and stay below 23,170 rows."""
    p = W.config2()
    prob = pk.Problem.from_workload(p)
    with pytest.raises(pk.BDDCSOError) as e:
        prob.plan_stats(coarse_solver=1)
    assert e.value.name == "EINVAL" and "4 GiB" in str(e.value)
    with pytest.raises(pk.BDDCSOError):
        prob.workspace_size(coarse_solver=1)
    st = prob.plan_stats(coarse_solver=0)
    assert st["n_coarse"] == 39823 and st["max_front"] < 23170


def test_vertex_free_floating_subdomain_is_planned():
    """A primal set without point constraints leaves the subdomains that do
    not touch the Dirichlet boundary with constants in the kernel of their
    local matrices: the planner pins one interior node of each (and carries
    the constant separately) instead of refusing the set."""
    p = W.config2_like(n=18, H=6, L=3, log_range=None)   # 3^3 subdomains: the centre one floats
    prob = pk.Problem.from_workload(p)
    for mask in range(1, 8):
        assert prob.plan_stats(primal_mask=mask)["n_coarse"] > 0
    c = W.channels_problem(n=24, subs=3, ell=6, per_axis=1)
    assert pk.Problem.from_workload(c).plan_stats(primal_mask=4)["n_coarse"] == 60
