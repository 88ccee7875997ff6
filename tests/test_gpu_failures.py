"""Numerical failure paths of gks_run, forced from the host (every kernel still exits normally).

  * A NaN planted in the initial state makes the recorded energy non-finite: gks_run returns
    GKS_ENONFINITE, names the step of the first bad record, and stops there instead of running
    every step (the records after the stopping point are not written).
  * A point source that pumps energy into an empty box makes the energy grow past the
    unstable_growth factor: GKS_EUNSTABLE, with the same early stop; without the threshold the
    same run completes.
  * 3D grids refuse Courant numbers above 1/3 at init, before any launch (the D3Q4 step grows
    there); the library's own test of that is on the CPU (test_abi.py), this one goes through the
    Python binding.
"""
import numpy as np
import pytest

from paper_2412_16845_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


def dev(torch, a, precision):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if precision == "fp64" else torch.float32,
                        device="cuda")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("every", [1, 5])
def test_nan_state_stops_with_enonfinite(torch, precision, every):
    from paper_2412_16845_amd.gks import GKSError, Solver
    wl = I.tm_dielectric_nr(nx=96, ny=80, seed=3, nsteps=0, ncircles=6, pulse=1.0)
    s = Solver("cart2d", n=wl.n, bc=wl.bc, precision=precision, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt,
               energy_every=every)
    s.set_material(dev(torch, wl.epsinv, precision))
    U = dev(torch, wl.U0, precision)
    U[0, 1, 40, 50] = float("nan")
    nsteps = 200
    rec = np.full((nsteps // every, 1), -7.0)
    from paper_2412_16845_amd import gks as G
    st = G.lib().gks_run(s._h, U.data_ptr(), nsteps, 0.0, rec.ctypes.data)
    msg = G.lib().gks_last_error(s._h).decode()
    assert st == -5, (st, msg)                     # GKS_ENONFINITE
    assert f"after step {every}" in msg, msg       # the first record is already bad
    assert np.isnan(rec[0, 0])
    # stopped early: at most the record after the failing one was written
    assert np.all(rec[2:] == -7.0), rec[:4].ravel()
    # the same through the Python binding, which raises
    V = dev(torch, wl.U0, precision)
    V[0, 0, 10, 10] = float("inf")
    with pytest.raises(GKSError, match="ENONFINITE"):
        s.run(V, 20, energy=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_growing_energy_stops_with_eunstable(torch, precision):
    from paper_2412_16845_amd import gks as G
    from paper_2412_16845_amd.gks import Solver
    wl = I.tm_dielectric_nr(nx=64, ny=64, seed=5, nsteps=0, ncircles=4)   # empty box, source at the centre
    src = wl.source
    every, nsteps = 2, 400
    results = {}
    for growth in (10.0, 0.0):
        s = Solver("cart2d", n=wl.n, bc=wl.bc, precision=precision, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt,
                   energy_every=every, unstable_growth=growth)
        s.set_material(dev(torch, wl.epsinv, precision))
        s.set_point_source(src["cells"], src["weights"], src["J0"], src["t0"], src["sigma_t"])
        U = dev(torch, wl.U0, precision)
        rec = np.full((nsteps // every, 1), -7.0)
        st = G.lib().gks_run(s._h, U.data_ptr(), nsteps, 0.0, rec.ctypes.data)
        results[growth] = (st, G.lib().gks_last_error(s._h).decode(), rec)
    st, msg, rec = results[10.0]
    assert st == -4, (st, msg)                     # GKS_EUNSTABLE
    assert "grew by" in msg
    k = int(msg.rsplit("after step", 1)[1]) // every - 1    # the failing record
    assert np.all(rec[:k] <= 10.0 * rec[0]) and rec[k, 0] > 10.0 * rec[0, 0]
    assert np.all(rec[k + 2:] == -7.0)            # stopped at most one record later
    st0, msg0, rec0 = results[0.0]
    assert st0 == 0, msg0                          # no threshold: the whole run, every record
    assert np.all(rec0 > 0.0) and np.array_equal(rec0[:k + 1], rec[:k + 1])


def test_3d_courant_above_one_third_is_refused(torch):
    from paper_2412_16845_amd.gks import GKSError, Solver
    with pytest.raises(GKSError, match="1/3"):
        Solver("cart3d", n=(16, 16, 16), bc=("pec",) * 6, cfl=0.5)
    s = Solver("cart3d", n=(16, 16, 16), bc=("pec",) * 6, cfl=1.0 / 3.0)
    assert abs(s.dt - (1.0 / 3.0) / 16) <= 1e-16
