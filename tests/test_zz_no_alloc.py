"""The allocation-free adaptive step (pa_adaptive_dbeta_noalloc) against the
handle entry point pa_adaptive_dbeta on the same populations: two calls in a
row, the second with a smaller population (the scratch array still holds the
first call's histogram), then one of a smaller lattice."""
import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2102_06611_amd as pa
from workloads import linear_schedule

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pa.lib()


def _handle_answer(L, R, steps, first, count, seed=31):
    """pa_adaptive_dbeta and pa_overlap of replicas [first, first + count) of a
    run after `steps` steps (adopted by a second handle when not the whole
    population), with their energies."""
    betas = linear_schedule(0.44, 20)
    run = pa.Run(L, R, betas, 3, seed, "nearest", "msc64")
    run.run(steps)
    spins, fam, E, _ = run.population()
    _, R_i = run.current()
    if count < R_i:
        sub = pa.Run(L, R, betas, 3, seed, "nearest", "msc64")
        sub.set_population(steps, spins[first:first + count], fam[first:first + count],
                           run.observables(steps)["minus_beta_F"])
        run.close()
        run = sub
    d = run.adaptive_dbeta(0.85, 0.5)
    a = run.overlap(d)
    run.close()
    return d, a, np.ascontiguousarray(E[first:first + count])


def test_noalloc_adaptive_step_matches_the_handle_entry_point():
    s = torch.cuda.Stream()
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    cases = [(16, 3000, 8, 0, 3000), (16, 3000, 8, 500, 1200), (8, 700, 5, 0, 700)]
    for L, R, steps, first, count in cases:
        d, a, E = _handle_answer(L, R, steps, first, count)
        if count == R:
            assert len(E) >= R - 200  # the whole population of the step
        E_dev = torch.from_numpy(E).cuda()
        pa.adaptive_dbeta_noalloc(E_dev, L, 0.85, 0.5, out, stream=s)
        s.synchronize()
        got = out.cpu().numpy()
        assert got[0] == d, (L, count, got[0], d)   # same histogram, same search
        assert abs(got[1] - a) < 1e-9 and got[1] >= 0.85 - 1e-9, (got[1], a)


def test_noalloc_rejects_what_its_scratch_cannot_hold():
    E = torch.zeros(4, dtype=torch.int32, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    L = pa.lib()
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.pa_adaptive_dbeta_noalloc(P(E), 4, 130, 0.85, 0.5, P(out), None) == pa.PA_ERR_ARG
    assert L.pa_adaptive_dbeta_noalloc(P(E), 4, 7, 0.85, 0.5, P(out), None) == pa.PA_ERR_ARG
    assert L.pa_adaptive_dbeta_noalloc(P(E), 0, 8, 0.85, 0.5, P(out), None) == pa.PA_ERR_ARG
    assert L.pa_adaptive_dbeta_noalloc(P(E), 4, 8, 1.5, 0.5, P(out), None) == pa.PA_ERR_ARG
    assert L.pa_adaptive_dbeta_noalloc(P(E), 4, 8, 0.85, float("inf"), P(out), None) == pa.PA_ERR_ARG
    assert pa.lib().pa_last_error(None)
    # an energy that no 8 x 8 torus has gives NaN, not a histogram write
    bad = torch.tensor([0, 4, 1, -128], dtype=torch.int32, device="cuda")
    pa.adaptive_dbeta_noalloc(bad, 8, 0.85, 0.5, out)
    torch.cuda.synchronize()
    assert all(math.isnan(x) for x in out.cpu().numpy())
