"""Many-instance solves (ommSolveBatched): every instance, solved beside the others on its own
stream, gives exactly the result it gives alone, at the oracle's energy."""

import numpy as np
import pytest

from oracle import hamiltonian as ham
from paper_1603_09724_amd import inputs
from tests.gpu_common import announce, to_gpu_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pomm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1603_09724_amd import pomm as p
    return p


def test_batched_equals_alone(pomm):
    import torch
    cases = [(1701, 32, 8), (1702, 48, 5), (1703, 32, 12), (1704, 48, 3), (1705, 32, 1)]
    insts, wins, lams = [], [], []
    for seed, m, N in cases:
        inst = inputs.small_2d(seed=seed, m=m, N=N)
        lam = np.linalg.eigvalsh(ham.dense_h(2, m, inst.V))
        insts.append(inst)
        lams.append(lam)
        wins.append((float(inst.V.min()), float(lam[N - 1]), float(lam[N])))
    streams = [torch.cuda.Stream() for _ in cases]
    handles = []
    for inst, win, st in zip(insts, wins, streams):
        with torch.cuda.stream(st):
            handles.append(pomm.Handle(2, inst.m, inst.V, inst.N, win, stream=st,
                                       options=pomm.default_options(filter_rtol=1e-10, gmres_rtol=1e-8)))
    torch.cuda.synchronize()
    X0 = [to_gpu_block(inst.X0) for inst in insts]
    alone = []
    for h, x in zip(handles, X0):
        X = x.clone()
        torch.cuda.synchronize()
        info = h.solve(X)
        alone.append((X, info))
    announce("alone: " + " ".join("%d" % a[1]["iters"] for a in alone))
    Xs = [x.clone() for x in X0]
    torch.cuda.synchronize()
    infos = pomm.solve_batched(handles, Xs)
    torch.cuda.synchronize()
    for k, (inst, lam) in enumerate(zip(insts, lams)):
        assert infos[k]["status"] == pomm.OK
        assert torch.equal(Xs[k], alone[k][0])
        assert infos[k]["iters"] == alone[k][1]["iters"]
        Estar = 0.5 * np.sum(lam[:inst.N] - handles[k].sigma)
        assert abs(infos[k]["energy"] - Estar) <= 1e-10 * abs(Estar)
    announce("batched: " + " ".join("%d" % i["iters"] for i in infos))
    for h in handles:
        h.close()


def test_batched_rejects_repeated_handles(pomm):
    inst = inputs.small_2d(m=16, N=2)
    lam = np.linalg.eigvalsh(ham.dense_h(2, 16, inst.V))
    h = pomm.Handle(2, 16, inst.V, 2, (float(inst.V.min()), float(lam[1]), float(lam[2])))
    X = to_gpu_block(inst.X0)
    with pytest.raises(pomm.PommError) as e:
        pomm.solve_batched([h, h], [X, X.clone()])
    assert e.value.code == pomm.EINVAL
    h.close()
