"""GPU parity of the comparison preconditioners of Section 3.1 (inverse shifted Laplacian and
TPA, opts.outer) against the oracle, and Algorithm 1 with them (the paper's contrast)."""

import numpy as np
import pytest

from oracle import comparison as cmp, hamiltonian as ham, metrics, omm
from paper_1603_09724_amd import inputs
from tests.gpu_common import announce, from_gpu_block, rel, to_gpu_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pomm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1603_09724_amd import pomm as p
    return p


def _window(inst):
    lam, U = np.linalg.eigh(ham.dense_h(2, inst.m, inst.V))
    return lam, U, (float(np.min(inst.V)), float(lam[inst.N - 1]), float(lam[inst.N]))


@pytest.mark.parametrize("m", [32, 48])
@pytest.mark.parametrize("kind", ["laplace", "tpa"])
def test_outer_apply_matches_oracle(pomm, m, kind):
    import torch
    announce("outer %s m=%d" % (kind, m))
    inst = inputs.small_2d(m=m, N=4)
    lam, U, win = _window(inst)
    outer = pomm.OUTER_LAPLACE if kind == "laplace" else pomm.OUTER_TPA
    h = pomm.Handle(2, m, inst.V, inst.N, win, options=pomm.default_options(outer=outer, tau=3.7))
    G = to_gpu_block(inst.X0)
    PG = torch.empty_like(G)
    h.precondition(G, PG)
    torch.cuda.synchronize()
    sym = cmp.laplace_symbol(2, m, 3.7) if kind == "laplace" else cmp.tpa_symbol(2, m, 3.7)
    assert rel(from_gpu_block(PG), cmp.apply(2, m, sym, inst.X0)) < 1e-13
    h.close()


def test_tpa_solve_reaches_minimum_slowly(pomm):
    """Algorithm 1 with TPA (tau by Section 4's rule) reaches the energy of eigh's N lowest
    eigenvalues to 1e-10, in more than three times the iterations of the Fermi projection."""
    import torch
    inst = inputs.small_2d()
    lam, U, win = _window(inst)
    N = inst.N
    tau = cmp.tau_rule(2, inst.m, U[:, :N])
    runs = {}
    for kind, opts in (("fermi", dict(filter_rtol=1e-10, gmres_rtol=1e-8)),
                       ("tpa", dict(outer=pomm.OUTER_TPA, tau=tau))):
        announce("solve well4 m=32 N=8 with %s" % kind)
        h = pomm.Handle(2, inst.m, inst.V, N, win, options=pomm.default_options(**opts))
        Xg = to_gpu_block(inst.X0)
        info = h.solve(Xg)
        torch.cuda.synchronize()
        X = from_gpu_block(Xg)
        E = omm.energy(X, ham.apply_h(2, inst.m, inst.V, X, h.sigma))
        Estar = 0.5 * np.sum(lam[:N] - h.sigma)
        announce("%s: iters=%d rule=%s E_rel=%.2e" % (kind, info["iters"], info["stop_rule"],
                                                       abs(E - Estar) / abs(Estar)))
        assert info["status"] == pomm.OK
        assert abs(E - Estar) <= 1e-10 * abs(Estar)
        runs[kind] = info["iters"]
        h.close()
    assert runs["tpa"] > 3 * runs["fermi"]


def test_outer_needs_positive_tau(pomm):
    inst = inputs.small_2d(m=16, N=2)
    lam, U, win = _window(inst)
    with pytest.raises(pomm.PommError) as e:
        pomm.Handle(2, 16, inst.V, 2, win, options=pomm.default_options(outer=pomm.OUTER_TPA))
    assert e.value.code == pomm.EINVAL
