"""The allocation-free H|psi> entry point (qm_apply_h_noalloc) against qm_apply_h, through the
C ABI, on two calls in a row, the second with a smaller input.

Bound: float64, per-band relative difference <= 1e-12 (the local part is the same kernels on
the same bands; the projector GEMM sums a chunk of bands with a different split-K schedule,
so only the order of float64 additions differs).  The 64-atom cell with two k-points and
160 bands needs three band chunks per k-point in the 64 MiB scratch array; the second call
(k = 1 alone, 37 bands) reuses the array that the first call left filled.  The 2-atom cell
is also checked against the oracle."""
import numpy as np
import pytest

import workload
from oracle import hamiltonian as ham
from hpsi_inputs import band_rel_err, make_plan, psi_block, split_k

pytestmark = pytest.mark.gpu


def _both(plan, k, psi_np, nbnd):
    import torch
    import paper_2308_07277_amd as qm
    x = torch.from_numpy(psi_np).cuda()
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, complex(np.nan, np.nan))
    qm.qm_apply_h(plan, k, x, y_ref, nbnd)
    qm.qm_apply_h_noalloc(plan, k, x, y_na, nbnd)
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


@pytest.mark.parametrize("prec,bound", [(0, 1e-12), (1, 1e-5)])
def test_noalloc_matches_apply_h_two_calls(prec, bound):
    w = workload.make_workload("c3", nk_limit=2)
    plan, a = make_plan(w, w.nbnd, prec=prec)
    flat, per = psi_block(w, w.nbnd)
    ref, got = _both(plan, -1, flat, w.nbnd)
    r, g = split_k(ref, w, w.nbnd), split_k(got, w, w.nbnd)
    err = max(band_rel_err(g[ik], r[ik]).max() for ik in range(w.nk))
    print(f"prec {prec} call 1 (2 k x 160 bands): max per-band rel diff {err:.2e}")
    assert np.isfinite(got).all() and err <= (1e-12 if prec == 0 else 1e-6)
    # second call: smaller input, one k-point, 37 bands
    nb = 37
    x1 = w.psi(1, purpose=3, nbnd=nb)
    ref1, got1 = _both(plan, 1, x1.reshape(-1).copy(), nb)
    err1 = band_rel_err(got1.reshape(nb, -1), ref1.reshape(nb, -1)).max()
    print(f"prec {prec} call 2 (k=1, {nb} bands): max per-band rel diff {err1:.2e}")
    assert np.isfinite(got1).all() and err1 <= (1e-12 if prec == 0 else 1e-6)
    # and the oracle on sampled bands of the second call
    m = w.miller[1]
    off = int(w.npw[0]) * w.nproj
    beta = a["beta"][off:off + w.nproj * m.shape[0]].reshape(w.nproj, m.shape[0])
    o = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[1], m, a["vloc"], beta, a["dmat"], x1[[0, 36]])
    assert band_rel_err(got1.reshape(nb, -1)[[0, 36]], o).max() <= bound
    plan.close()


def test_noalloc_small_cell_vs_oracle_and_errors():
    import torch
    import paper_2308_07277_amd as qm
    w = workload.make_workload("c1")
    plan, a = make_plan(w, w.nbnd)
    flat, per = psi_block(w, w.nbnd)
    ref, got = _both(plan, 0, flat, w.nbnd)
    o = ham.apply_h_ref(w.cell, w.grid, w.k_cryst[0], w.miller[0], a["vloc"],
                        a["beta"].reshape(w.nproj, -1), a["dmat"], per[0])
    assert band_rel_err(got.reshape(w.nbnd, -1), o).max() <= 1e-12
    x = torch.from_numpy(flat).cuda()
    with pytest.raises(qm.QmError) as e:
        qm.qm_apply_h_noalloc(plan, 0, x, x, w.nbnd)
    assert e.value.code == qm.QM_E_ARG
    with pytest.raises(qm.QmError) as e:
        qm.qm_apply_h_noalloc(plan, 1, x, torch.empty_like(x), w.nbnd)
    assert e.value.code == qm.QM_E_ARG
    plan.close()
