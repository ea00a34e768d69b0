"""The allocation-free band-to-full entry point (trans_ev_band_to_full_z_noalloc)
against the workspace form trans_ev_band_to_full_z through the C ABI: the
same kernels, so the results must agree bit for bit (and so within the
1e-12 relative Frobenius bound of the parity tests).  Two calls in a row on
one stream, the second on a smaller problem, so the fixed scratch still
holds the first call's factors when the second starts."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _inputs(n, nbw, nev, seed):
    import torch
    import synth
    V, tau = synth.full_unitary_reflectors(n, nbw, seed, "z")
    Y = synth.gaussian(n, nev, seed + 1, "z")
    ldv, ldz = n + 3, n + 1
    J = V.shape[1]
    hv = np.zeros((J, ldv), np.complex128)
    hv[:, :n] = V.T
    zb = np.full((nev, ldz), 5.0 + 5.0j)
    zb[:, :n] = Y.T
    dev = torch.device("cuda:0")
    return (torch.from_numpy(hv).to(dev), torch.from_numpy(tau).to(dev),
            torch.from_numpy(zb).to(dev), ldv, ldz)


def test_noalloc_equals_workspace_form_two_calls():
    import torch
    import paper_2002_10991_amd as T
    for n, nbw, nev, seed in ((1500, 64, 300, 61), (700, 32, 90, 71)):
        print(f"[gpu] band_to_full_z_noalloc n={n} nbw={nbw} nev={nev}", flush=True)
        hv, tau, z0, ldv, ldz = _inputs(n, nbw, nev, seed)
        za, zb = z0.clone(), z0.clone()
        nb = T.trbt_band_to_full_workspace_bytes(n, nbw, nev, True)
        buf = torch.empty(nb + 256, dtype=torch.uint8, device="cuda:0")
        work = buf[(-buf.data_ptr()) % 256:][:nb]
        assert T.trans_ev_band_to_full_z(n, nbw, nev, hv, ldv, tau, za, ldz, work, nb) == 0
        assert T.trans_ev_band_to_full_z_noalloc(n, nbw, nev, hv, ldv, tau, zb, ldz) == 0
        torch.cuda.synchronize()
        a, b = za.cpu().numpy(), zb.cpu().numpy()
        assert np.all(b[:, n:] == 5.0 + 5.0j)          # rows n .. ldz-1 untouched
        err = np.linalg.norm(b - a) / np.linalg.norm(a)
        print(f"[gpu] noalloc vs workspace form: rel err {err:.2e}", flush=True)
        assert err <= 1e-12
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
        assert not np.array_equal(a[:, :n], z0.cpu().numpy()[:, :n])   # Z was transformed

