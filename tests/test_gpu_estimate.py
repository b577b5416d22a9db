"""GPU spectral window estimate (ommEstimateSpectrum) against the exact spectrum: the
oracle's dense eigh (small grids) and the stored spectrum (128x128).  The window is the
spectral information Section 4 builds the contour from."""

import numpy as np
import pytest

from oracle import hamiltonian as ham, omm
from paper_1603_09724_amd import inputs
from tests.gpu_common import announce, from_gpu_block, load_spectra, to_gpu_block

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def pomm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1603_09724_amd import pomm as p
    return p


def _real_block(n, cols, seed):
    import torch
    B = inputs.gaussian_test_block(n, cols, seed)
    return torch.from_numpy(np.ascontiguousarray(B.T)).to("cuda:0")


def _check_window(est, V, lam, N):
    """Interlacing: theta_N >= lambda_N; |theta - lambda| <= residual <= tol max(1, |theta|);
    lumo = theta_{N+1} - res_{N+1} <= lambda_{N+1}; lo = min V."""
    scale_h, scale_l = max(1.0, abs(lam[N - 1])), max(1.0, abs(lam[N]))
    assert est["converged"]
    assert est["lo"] == float(np.min(V))
    assert est["homo"] >= lam[N - 1] - 1e-12 * scale_h
    assert est["homo"] - lam[N - 1] <= TOL * scale_h
    assert est["lumo"] <= lam[N] + 1e-12 * scale_l
    assert lam[N] - est["lumo"] <= 2 * TOL * scale_l
    assert est["res_homo"] <= TOL * scale_h and est["res_lumo"] <= TOL * scale_l


@pytest.mark.parametrize("m,N,extra", [(32, 8, 8), (48, 12, 4)])
def test_estimate_small_2d(pomm, m, N, extra):
    announce("estimate 2D m=%d N=%d block %d" % (m, N, N + extra))
    inst = inputs.small_2d(m=m, N=N)
    lam = np.linalg.eigvalsh(ham.dense_h(2, m, inst.V))
    est = pomm.estimate_spectrum(2, m, inst.V, N, _real_block(inst.n, N + extra, 31), tol=TOL)
    announce("iters=%d applies=%d homo %.12f (exact %.12f) lumo %.12f (exact %.12f)" % (
        est["iters"], est["applies"], est["homo"], lam[N - 1], est["lumo"], lam[N]))
    _check_window(est, inst.V, lam, N)


def test_estimate_3d(pomm):
    announce("estimate 3D m=16 N=8")
    inst = inputs.lattice_3d(m=16, N=8)
    lam = np.linalg.eigvalsh(ham.dense_h(3, 16, inst.V))
    est = pomm.estimate_spectrum(3, 16, inst.V, 8, _real_block(inst.n, 16, 32), tol=TOL)
    announce("iters=%d applies=%d homo %.12f (exact %.12f) lumo %.12f (exact %.12f)" % (
        est["iters"], est["applies"], est["homo"], lam[7], est["lumo"], lam[8]))
    _check_window(est, inst.V, lam, 8)


def test_estimate_lattice128_and_solve(pomm):
    """128x128, N = 64, 72 columns: the window against the stored spectrum, then the timed
    mixed solve on that window reaches the exact minimum energy to 1e-10."""
    import torch
    rec = load_spectra().get("lattice8_2d_m128_N64")
    if rec is None:
        pytest.skip("spectra.json has no 128x128 record")
    announce("estimate lattice8 m=128 N=64")
    inst = inputs.lattice_2d()
    lam = np.array(rec["lambda"])
    N = inst.N
    est = pomm.estimate_spectrum(2, 128, inst.V, N, _real_block(inst.n, N + 8, 1607), tol=TOL)
    announce("iters=%d applies=%d homo %.12f (stored %.12f) lumo %.12f (stored %.12f)" % (
        est["iters"], est["applies"], est["homo"], lam[N - 1], est["lumo"], lam[N]))
    _check_window(est, inst.V, lam, N)
    h = pomm.Handle(2, 128, inst.V, N, (est["lo"], est["homo"], est["lumo"]),
                    options=pomm.default_options(precision=pomm.MIXED, gmres_rtol=5e-4, filter_rtol=1e-5,
                                                 npoles=30))
    Xg = to_gpu_block(inst.X0)
    info = h.solve(Xg)
    torch.cuda.synchronize()
    X = from_gpu_block(Xg)
    Estar = 0.5 * np.sum(lam[:N] - h.sigma)
    E = omm.energy(X, ham.apply_h(2, 128, inst.V, X, h.sigma))
    announce("solve on the estimated window: iters=%d E_rel=%.2e" % (info["iters"], abs(E - Estar) / abs(Estar)))
    assert info["status"] == pomm.OK
    assert abs(E - Estar) <= 1e-10 * abs(Estar)
    h.close()


def test_estimate_rejects_bad_sizes(pomm):
    inst = inputs.small_2d()
    for cols in (inst.N, inst.N + 1):
        with pytest.raises(pomm.PommError) as e:
            pomm.estimate_spectrum(2, 32, inst.V, inst.N, _real_block(inst.n, cols, 3))
        assert e.value.code == pomm.EINVAL


@pytest.mark.parametrize("precision", [0, 1])
def test_setup_without_window(pomm, precision):
    """ommSetup with no window estimates it (SplitMix64 start block): the window brackets
    the exact gap, and the solve on it reaches the exact minimum energy to 1e-10."""
    import torch
    announce("setup without a window, well4 m=32 N=8, precision=%d" % precision)
    inst = inputs.small_2d()
    N = inst.N
    lam = np.linalg.eigvalsh(ham.dense_h(2, 32, inst.V))
    opts = pomm.default_options(precision=precision)
    if precision == 1:
        opts = pomm.default_options(precision=precision, filter_rtol=1e-7, gmres_rtol=1e-6)
    h = pomm.Handle(2, 32, inst.V, N, None, options=opts)
    lo, homo, lumo = h.spectrum()
    announce("window lo %.6f homo %.12f (exact %.12f) lumo %.12f (exact %.12f)" % (lo, homo, lam[N - 1], lumo,
                                                                                  lam[N]))
    assert lo == float(np.min(inst.V))
    assert lam[N - 1] - 1e-12 <= homo <= lam[N - 1] + TOL * max(1.0, abs(lam[N - 1]))
    assert lam[N] - 2 * TOL * max(1.0, abs(lam[N])) <= lumo <= lam[N] + 1e-12
    Xg = to_gpu_block(inst.X0)
    info = h.solve(Xg)
    torch.cuda.synchronize()
    X = from_gpu_block(Xg)
    Estar = 0.5 * np.sum(lam[:N] - h.sigma)
    E = omm.energy(X, ham.apply_h(2, 32, inst.V, X, h.sigma))
    announce("iters=%d E_rel=%.2e" % (info["iters"], abs(E - Estar) / abs(Estar)))
    assert info["status"] == pomm.OK
    assert abs(E - Estar) <= 1e-10 * abs(Estar)
    h.close()
