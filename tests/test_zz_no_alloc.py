"""The allocation-free PGS entry point (icr_solve_contacts_noalloc) against
icr_solve_contacts, the entry point it is a variant of, and the FP64 oracle.

Both entry points run the same kernels, so their outputs must agree bit for
bit; the oracle's PGS (Eq. 18-19, Algorithm 1) is checked at 1e-10 with
identical sweep counts and classification.  Two calls in a row on the shared
static work array, the second with fewer contacts, show that a call does not
depend on what the previous one left there.
"""
import ctypes

import numpy as np
import pytest

import oracle.icr_oracle as O
from paper_2306_06946_amd.scenes import random_contact_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def _run_noalloc(L, stream, W, d, mu, h, lam, status, max_sweeps, tol, j_inner):
    sw, ep = ctypes.c_int32(0), ctypes.c_double(0.0)
    nc = mu.numel()
    code = L.icr_solve_contacts_noalloc(ctypes.c_void_p(stream), nc, W.data_ptr(), d.data_ptr(), mu.data_ptr(), h,
                                        lam.data_ptr(), status.data_ptr(), max_sweeps, tol, j_inner,
                                        ctypes.byref(sw), ctypes.byref(ep))
    return code, sw.value, ep.value


def test_noalloc_pgs_equals_the_scene_entry_point_twice():
    from paper_2306_06946_amd import icr
    L = icr.lib()
    scene = icr.Scene()
    stream = torch.cuda.current_stream().cuda_stream
    h = 0.01
    for nc, seed, sweeps in ((1000, 71, 30), (150, 72, 60)):
        rng = np.random.default_rng(seed)
        W, d, mu, lam0 = random_contact_problem(nc, rng)
        lam0[: 3 * (nc // 4)] = np.abs(rng.standard_normal(3 * (nc // 4))) * 1e-3   # a warm start on a quarter
        Wd = torch.as_tensor(W.ravel()).cuda()
        dd = torch.as_tensor(d).cuda()
        mud = torch.as_tensor(mu).cuda()
        lam_a = torch.as_tensor(lam0).cuda()
        lam_b = lam_a.clone()
        st_a = torch.full((nc,), -1, dtype=torch.int8, device="cuda")
        st_b = st_a.clone()
        _say(f"[gpu] noalloc PGS nc={nc}")
        code, sw_b, ep_b = _run_noalloc(L, stream, Wd, dd, mud, h, lam_b, st_b, sweeps, 1e-12, 8)
        assert code in (icr.OK, icr.WARN_NOT_CONVERGED), code
        _say(f"[gpu] scene PGS nc={nc}")
        sw_a, ep_a = scene.solve_contacts(Wd, dd, mud, h, lam_a, st_a, sweeps, 1e-12, 8)
        torch.cuda.synchronize()
        assert sw_b == sw_a and ep_b == ep_a
        assert torch.equal(lam_a, lam_b) and torch.equal(st_a, st_b)
        lam_ref, st_ref, sw_ref, _ = O.pgs(W, d, mu, h, lam0, sweeps, 1e-12, 8)
        assert sw_b == sw_ref
        assert np.array_equal(st_b.cpu().numpy(), st_ref)
        assert _rel(lam_b.cpu().numpy(), lam_ref) <= 1e-10
    scene.close()


def test_noalloc_pgs_refuses_what_it_cannot_hold():
    from paper_2306_06946_amd import icr
    L = icr.lib()
    buf = torch.zeros(16, dtype=torch.float64, device="cuda")
    st8 = torch.zeros(16, dtype=torch.int8, device="cuda")
    p = buf.data_ptr()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.icr_solve_contacts_noalloc(stream, 1025, p, p, p, 0.01, p, st8.data_ptr(), 3, 0.0, 8, None,
                                        None) == icr.E_ARG
    assert L.icr_solve_contacts_noalloc(stream, 0, p, p, p, 0.01, p, st8.data_ptr(), 3, 0.0, 8, None,
                                        None) == icr.E_ARG
    assert L.icr_solve_contacts_noalloc(stream, 4, p, p, p, float("nan"), p, st8.data_ptr(), 3, 0.0, 8, None,
                                        None) == icr.E_ARG
    assert L.icr_solve_contacts_noalloc(stream, 4, None, p, p, 0.01, p, st8.data_ptr(), 3, 0.0, 8, None,
                                        None) == icr.E_ARG
