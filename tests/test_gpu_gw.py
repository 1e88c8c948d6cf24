"""GW plane-wave matrix elements on the GPU against the FP64 oracle (oracle/gw.py).

Bound: element by element within 1e-12 of the largest |M| (three float64 3-D FFTs of
10^4-10^5 points per element)."""
import numpy as np
import pytest

import workload
from oracle import gw
from hpsi_inputs import make_plan

pytestmark = pytest.mark.gpu


def _g_list(w, n):
    """The n shortest G of the k = 0 sphere of the workload (a q = 0 epsilon cutoff)."""
    m = w.miller[0]
    return m[:n]


@pytest.mark.parametrize("name,kq,k,nb1,nb2,ng", [("c1", 0, 0, 4, 6, 27), ("c2", 1, 0, 5, 7, 59),
                                                   ("c2", 2, 2, 3, 3, 200)])
def test_mtxel_vs_oracle(name, kq, k, nb1, nb2, ng):
    import torch
    import paper_2308_07277_amd as qm
    w = workload.make_workload(name)
    plan, a = make_plan(w, max(nb1, nb2))
    ckq = w.psi(kq, purpose=5, nbnd=nb1)
    ck = w.psi(k, purpose=6, nbnd=nb2)
    mg = _g_list(w, ng)
    out = torch.empty((nb1, nb2, ng), dtype=torch.complex128, device="cuda")
    qm.qm_mtxel(plan, kq, torch.from_numpy(ckq.reshape(-1).copy()).cuda(), nb1, k,
                torch.from_numpy(ck.reshape(-1).copy()).cuda(), nb2, mg, out)
    ref = gw.mtxel_direct(ckq, w.miller[kq], ck, w.miller[k], mg)
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"{name} kq={kq} k={k}: max rel err {err:.2e}")
    assert err <= 1e-12


def test_mtxel_orthonormal_bands_give_identity_at_g0():
    import torch
    import paper_2308_07277_amd as qm
    w = workload.make_workload("c2")
    plan, a = make_plan(w, 6)
    q, _ = np.linalg.qr(w.psi(3, nbnd=6).T)
    c = torch.from_numpy(np.ascontiguousarray(q.T).reshape(-1)).cuda()
    out = torch.empty((6, 6, 1), dtype=torch.complex128, device="cuda")
    qm.qm_mtxel(plan, 3, c, 6, 3, c, 6, np.zeros((1, 3), np.int32), out)
    np.testing.assert_allclose(out.cpu().numpy()[:, :, 0], np.eye(6), atol=1e-13)
