"""fk_build_jk_noalloc (the build in the library's fixed scratch array, no
allocation) against fk_build_jk on the same context, through the C ABI: two
calls in a row, the second with a smaller input, each within 1e-12 of the
allocating build (the two differ only in the order of the FP64 atomic adds:
one accumulator copy instead of one per XCD) and, for the small unscreened
case, within 1e-10 of the oracle.  Run with -m gpu."""
import numpy as np
import pytest

import oracle
from oracle.scf import core_guess, orthogonalizer
from synth import workloads as wl

pytestmark = pytest.mark.gpu


def _core_D(s):
    S, T, V = oracle.oneel(s)
    return core_guess(T + V, orthogonalizer(S), s["nelec"] // 2)


def test_noalloc_equals_build_jk():
    import torch
    import paper_2407_21445_amd as fk
    assert torch.cuda.is_available()
    cases = [(wl.c20h42_631gs(), 1e-10, 1e-12), (wl.water4_sto3g(), 0.0, 0.0)]
    for s, tau, tau_prim in cases:
        c = fk.FockJK(0).set_system(s).build_quartets(tau=tau, tau_prim=tau_prim)
        D = _core_D(s)
        Dd = torch.tensor(D, dtype=torch.float64, device="cuda")
        J0, K0 = c.build_jk(Dd, sync=True)
        J0, K0 = J0.clone(), K0.clone()
        J1 = torch.full_like(Dd, float("nan"))
        K1 = torch.full_like(Dd, float("nan"))
        c.build_jk_noalloc(Dd, J1, K1, sync=True)
        scale = max(1.0, float(J0.abs().max()))
        ej = float((J1 - J0).abs().max())
        ek = float((K1 - K0).abs().max())
        print(f"noalloc {s['name']}: max|dJ| {ej:.2e} max|dK| {ek:.2e}", flush=True)
        assert ej <= 1e-12 * scale and ek <= 1e-12 * scale
        assert c.stats()["quartets"] > 0
        # one matrix only (its own density screen): equal to fk_build_jk's J-only
        # build, the other argument untouched
        Jj, _ = c.build_jk(Dd, sync=True, only="J")
        J2 = torch.full_like(Dd, float("nan"))
        sentinel = torch.full_like(Dd, 3.0)
        c.build_jk_noalloc(Dd, J2, sentinel, sync=True, only="J")
        assert float((J2 - Jj).abs().max()) <= 1e-12 * scale
        assert bool(torch.all(sentinel == 3.0))
        if tau == 0:
            Jo, Ko = oracle.jk(s, D)
            assert np.max(np.abs(J1.cpu().numpy() - Jo)) <= 1e-10
            assert np.max(np.abs(K1.cpu().numpy() - Ko)) <= 1e-10
        c.close()


def test_noalloc_rejects_large_and_host_pointers():
    import torch
    import paper_2407_21445_amd as fk
    s = wl.water64_ccpvdz()   # 1600 functions: 2.56e6 matrix elements, above the scratch limit
    c = fk.FockJK(0).set_system(s).build_quartets(tau=1e-10, tau_prim=1e-12)
    D = torch.zeros((s["nbf"], s["nbf"]), dtype=torch.float64, device="cuda")
    J, K = torch.empty_like(D), torch.empty_like(D)
    with pytest.raises(fk.FockJKError) as e:
        c.build_jk_noalloc(D, J, K, sync=True)
    assert e.value.code == fk.FK_ERR_ARG and "scratch" in str(e.value)
    c.close()
