"""dwp_forces_noalloc, the allocation-free variant of dwp_forces, against
dwp_forces itself: the same kernels, with the packed atoms, the force partial
sums and the device copy of dE/dR in a static device array instead of context
buffers.  Two calls in a row, the second on a smaller input (a smaller grid,
fewer atoms), each compared with dwp_forces on the same state."""
import numpy as np
import pytest

from paper_0904_4887_amd import workloads as W

pytestmark = pytest.mark.gpu


def _solved(w, caller_eps=False):
    import torch
    from paper_0904_4887_amd.binding import Solver
    s = Solver(0)
    s.set_grid(w.n, w.L, z_wet_lo=w.z_wet[0], z_wet_hi=w.z_wet[1], tol=1e-10)
    if caller_eps:
        s.set_epsilon(torch.from_numpy(w.eps_grid()).cuda())
    else:
        s.build_epsilon(w.xyz, w.radius, w.eps_params)
    rho = s.build_rho(w.xyz, w.q, w.sigma)
    s.solve(rho)
    return s


def test_forces_noalloc_equals_forces_on_two_calls():
    from paper_0904_4887_amd.binding import DWPError, DWP_EINVAL
    # first call: 72 atoms, atom-built eps with the buried-atom height factor
    w = W.slab((48, 48, 96), exclusion=True)
    s = _solved(w)
    F_ref = s.forces(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
    F_na = s.forces_noalloc(w.xyz, w.q, w.sigma, w.radius, w.eps_params)
    assert np.array_equal(F_na, F_ref)
    s.close()
    # second call: a smaller input, 8 atoms on a 32 x 32 x 64 grid with a
    # caller-supplied eps (charge term only)
    t = W.tanh_box()
    s2 = _solved(t, caller_eps=True)
    F_ref2 = s2.forces(t.xyz, t.q, t.sigma)
    F_na2 = s2.forces_noalloc(t.xyz, t.q, t.sigma)
    assert np.array_equal(F_na2, F_ref2)
    assert np.abs(F_na2).max() > 0.0
    # an input larger than the static scratch is rejected before any device work
    n = 200_000
    rng = np.random.default_rng(0)
    xyz = rng.uniform(0.0, 10.0, size=(n, 3))
    with pytest.raises(DWPError) as e:
        s2.forces_noalloc(xyz, np.zeros(n), np.full(n, 0.5))
    assert e.value.status == DWP_EINVAL and "scratch" in e.value.message
    # the context is still usable afterwards
    assert np.array_equal(s2.forces_noalloc(t.xyz, t.q, t.sigma), F_ref2)
    s2.close()
