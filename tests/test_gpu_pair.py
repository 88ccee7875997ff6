"""The paired 2D kernel (two steps per launch) against single steps.

gks_run advances 2D TM grids (with or without psi) two steps per launch; its intermediate state
is the one a single step would store, and both stages do the single step's arithmetic in its
order.  So a run must equal the same number of gks_step calls bit for bit, on every side mix
(periodic sides included, with a source in the cell their ghosts image), with materials, a
point source, odd step counts and energy records that fall between two steps (where the run
takes single steps).  The oracle comparisons of the full-step tests run
through the same path.
"""
import numpy as np
import pytest

NR, PEC, PER = "nonreflecting", "pec", "periodic"

CASES = {
    # name: (nx, ny, bc, batch, eps, mu, source, nsteps, energy_every)
    "nr_box_source": ((300, 130), (NR,) * 4, 1, True, False, True, 7, 0),
    "mixed_mu_batch": ((257, 64), (PEC, NR, NR, PEC), 2, True, True, True, 10, 0),
    "pec_box_vacuum": ((131, 9), (PEC,) * 4, 1, False, False, False, 5, 0),
    "records_between": ((64, 300), (NR, PEC, PEC, NR), 3, True, False, True, 9, 3),
    "narrow": ((5, 40), (PEC, NR, PEC, NR), 2, True, True, False, 6, 0),
    "two_columns": ((2, 8), (NR,) * 4, 1, True, False, False, 4, 0),
    "strip_edges": ((245, 77), (NR, PEC, NR, PEC), 1, False, True, True, 8, 0),
    "periodic_x": ((70, 50), (PER, PER, NR, NR), 1, True, False, True, 6, 0),
    "periodic_y_pec_x": ((90, 33), (PEC, PEC, PER, PER), 2, True, True, True, 7, 0),
    "periodic_both_small": ((3, 9), (PER,) * 4, 1, True, False, True, 5, 0),
    "periodic_source_at_wrap": ((61, 40), (PER,) * 4, 1, True, False, "wrap", 6, 0),
    # short items in a batch: band cuts land one row from a side and move
    "short_items_batch": ((33, 11), (NR, PEC, PEC, NR), 3, True, False, True, 5, 0),
    "rows_9_pec": ((120, 9), (PEC,) * 4, 2, False, True, False, 4, 0),
}
# the PHM fields (Ez, Hx, Hy, psi): name -> grid, sides, batch, eps, mu, source, steps, couplings
PHM_CASES = {
    "phm_nr_source": ((190, 70), (NR,) * 4, 1, True, False, True, 7, (0.0, 1.0)),
    "phm_mixed_batch": ((67, 45), (PEC, NR, NR, PEC), 2, True, True, False, 6, (0.5, 0.8)),
}


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a GPU"
    return _t


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_run_equals_single_steps(torch, case, precision):
    from paper_2412_16845_amd.gks import Solver
    (nx, ny), bc, batch, eps, mu, source, nsteps, every = CASES[case]
    rng = np.random.default_rng(list(CASES).index(case) + 100 * (precision == "fp32"))
    dtype = torch.float64 if precision == "fp64" else torch.float32
    s = Solver("cart2d", n=(nx, ny), bc=bc, precision=precision, batch=batch, cfl=0.5, tau_over_dt=0.01,
               energy_every=every)
    ei = torch.tensor(rng.uniform(0.25, 1.0, (batch, ny, nx)), dtype=dtype, device="cuda") if eps else None
    mi = torch.tensor(rng.uniform(0.5, 1.0, (batch, ny, nx)), dtype=dtype, device="cuda") if mu else None
    s.set_material(ei, mi)
    if source == "wrap":   # the corner cell, which periodic ghosts of the other sides image
        s.set_point_source([(ny - 1) * nx + nx - 1], [1.3], 1.0, 0.01, 0.004)
    elif source:
        s.set_point_source([(ny // 3) * nx + nx // 2], [1.3], 1.0, 0.01, 0.004)
    U0 = torch.tensor(rng.standard_normal((batch, 3, ny, nx)), dtype=dtype, device="cuda")
    t0 = 0.0037
    A = U0.clone()
    rec = s.run(A, nsteps, t0, energy=every > 0)
    B = U0.clone()
    for k in range(nsteps):
        B = s.step(B, t=t0 + k * s.dt)
    torch.cuda.synchronize()
    same = bool(torch.equal(A, B))
    diff = float((A - B).abs().max())
    print(f"{case} {precision}: run vs single steps, max |diff| = {diff:.3e}")
    assert same
    if every:
        # the records are those of the single steps' states
        C = U0.clone()
        for k in range(nsteps):
            C = s.step(C, t=t0 + k * s.dt)
            if (k + 1) % every == 0:
                assert np.array_equal(rec[(k + 1) // every - 1], s.energy(C))


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(PHM_CASES))
def test_phm_run_equals_single_steps(torch, case, precision):
    from paper_2412_16845_amd.gks import Solver
    (nx, ny), bc, batch, eps, mu, source, nsteps, phm = PHM_CASES[case]
    rng = np.random.default_rng(50 + list(PHM_CASES).index(case) + 100 * (precision == "fp32"))
    dtype = torch.float64 if precision == "fp64" else torch.float32
    s = Solver("cart2d", n=(nx, ny), bc=bc, precision=precision, batch=batch, cfl=0.42, tau_over_dt=0.01, phm=phm)
    ei = torch.tensor(rng.uniform(0.25, 1.0, (batch, ny, nx)), dtype=dtype, device="cuda") if eps else None
    mi = torch.tensor(rng.uniform(0.5, 1.0, (batch, ny, nx)), dtype=dtype, device="cuda") if mu else None
    s.set_material(ei, mi)
    if source:
        s.set_point_source([(ny // 2) * nx + nx // 3], [0.8], 1.0, 0.01, 0.004)
    U0 = torch.tensor(rng.standard_normal((batch, 4, ny, nx)), dtype=dtype, device="cuda")
    A = U0.clone()
    s.run(A, nsteps, 0.002)
    B = U0.clone()
    for k in range(nsteps):
        B = s.step(B, t=0.002 + k * s.dt)
    torch.cuda.synchronize()
    print(f"{case} {precision}: run vs single steps, max |diff| = {float((A - B).abs().max()):.3e}")
    assert bool(torch.equal(A, B))


# minmod-limited slopes: name -> grid, sides, batch, eps, source, steps
LIM_CASES = {
    "lim_nr_source": ((150, 60), (NR,) * 4, 1, True, True, 7),
    "lim_pec_periodic": ((64, 45), (PEC, PEC, PER, PER), 2, True, False, 6),
}


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(LIM_CASES))
def test_limited_run_equals_single_steps(torch, case, precision):
    from paper_2412_16845_amd.gks import Solver
    (nx, ny), bc, batch, eps, source, nsteps = LIM_CASES[case]
    rng = np.random.default_rng(70 + list(LIM_CASES).index(case) + 100 * (precision == "fp32"))
    dtype = torch.float64 if precision == "fp64" else torch.float32
    s = Solver("cart2d", n=(nx, ny), bc=bc, precision=precision, batch=batch, cfl=0.5, tau_over_dt=0.01,
               limiter="minmod")
    ei = torch.tensor(rng.uniform(0.25, 1.0, (batch, ny, nx)), dtype=dtype, device="cuda") if eps else None
    s.set_material(ei, None)
    if source:
        s.set_point_source([(ny // 2) * nx + nx // 4], [1.1], 1.0, 0.01, 0.004)
    # discontinuous data, where the limiter acts
    U0 = torch.tensor(np.sign(rng.standard_normal((batch, 3, ny, nx))), dtype=dtype, device="cuda")
    A = U0.clone()
    s.run(A, nsteps, 0.001)
    B = U0.clone()
    for k in range(nsteps):
        B = s.step(B, t=0.001 + k * s.dt)
    torch.cuda.synchronize()
    print(f"{case} {precision}: run vs single steps, max |diff| = {float((A - B).abs().max()):.3e}")
    assert bool(torch.equal(A, B))
