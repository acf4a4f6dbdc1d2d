"""GPU parity of the final-stage limiter at the extremes of its work queue.

The limiter decides every cell in a first pass and hands the cells that need
more work (troubled cells, cells whose positivity needs the point test, the
learned indicator's band) to a per-block queue processed in a second pass.
These cases fill that queue completely, leave it empty, and take only the
positivity path, on meshes whose cell count is not a multiple of the
256-cell block.  The reference is the oracle's TVB limiter with its
positivity fallback (Section 2.2 for where the limiter acts; the minmod test
and the limited P1 reconstruction follow the TVB limiter the paper uses).
Flags are compared where the oracle's decision margin is above 1e-9; limited
states to 1e-13 relative wherever the flags agree.
"""
import numpy as np
import pytest

import oracle as O
from paper_2307_06471_amd import workloads as W
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_06471_amd import crkdg
    return crkdg


def setup(K, nx, ny, k, equation, u, bc=(0, 0, 0, 0)):
    eqo = O.EQ_EULER if equation == "euler" else O.EQ_ADVECTION
    om = O.Mesh(2, nx, ny, bc=bc, equation=eqo, adv=(0.8, -0.6), flux=O.FLUX_LLF)
    lm = K.make_mesh(2, nx, ny, bc=bc, adv=(0.8, -0.6),
                     equation=K.EQ_EULER if equation == "euler" else K.EQ_ADVECTION)
    s = K.Solver(lm, k, K.FLUX_LLF, 3)
    s.crkdg_set_state(u)
    return om, s


def run_both(K, om, s, k, M, u):
    import torch
    flags = torch.zeros(om.ncells, dtype=torch.uint8, device="cuda")
    n_gpu = s.crkdg_limit(M, flags)
    lim_o, fl_o, n_o = O.limit_tvb(om, k, M, u)
    _, margin, _ = O.tvb_flags(om, k, M, u)
    return flags.cpu().numpy(), n_gpu, s.crkdg_get_state(), lim_o, fl_o, n_o, margin


def check(fg, n_gpu, got, lim_o, fl_o, n_o, margin, u):
    safe = margin > 1e-9
    assert np.array_equal(fg[safe], fl_o[safe])
    agree = fg == fl_o
    assert agree.mean() > 0.99
    assert rel_err(got[:, :, agree], lim_o[:, :, agree]) < 1e-13
    assert np.array_equal(got[:, 0], u[:, 0])  # cell averages untouched
    assert abs(n_gpu - n_o) <= (~safe).sum()


@pytest.mark.parametrize("k", [1, 2])
def test_every_cell_queued(K, k):
    """M = 0 on random modes: almost every cell is troubled, so the queue of
    every full block holds all 256 cells; 70 x 37 = 2590 cells leave a last
    block of 30"""
    nb = (k + 1) ** 2
    u = W.random_euler_modes(np.random.default_rng(40 + k), nb, 70 * 37)
    om, s = setup(K, 70, 37, k, "euler", u, bc=(1, 1, 1, 1))
    fg, n_gpu, got, lim_o, fl_o, n_o, margin = run_both(K, om, s, k, 0.0, u)
    print(f"[limiter] k={k} troubled {np.mean(fl_o & 1):.3f}", flush=True)
    assert np.mean(fl_o & 1) > 0.9
    check(fg, n_gpu, got, lim_o, fl_o, n_o, margin, u)


def test_positivity_path_only(K):
    """the TVB test never fires (M h^2 far above every jump) but large higher
    modes make density or pressure negative at quadrature points of some
    cells: those take the reconstruction (flag 2) and, if the limited P1
    polynomial still fails, drop to the average (flag 4)"""
    k, nx, ny = 2, 53, 29
    rng = np.random.default_rng(5)
    u = W.random_euler_modes(rng, 9, nx * ny, amp=0.25)
    om, s = setup(K, nx, ny, k, "euler", u)
    fg, n_gpu, got, lim_o, fl_o, n_o, margin = run_both(K, om, s, k, 1e12, u)
    print(f"[limiter] positivity flags 2: {np.mean(fl_o & 2 != 0):.3f} "
          f"4: {np.mean(fl_o & 4 != 0):.3f}", flush=True)
    assert not np.any(fl_o & 1)
    assert np.mean(fl_o & 2 != 0) > 0.05 and np.any(fl_o & 4)
    assert np.mean(fl_o == 0) > 0.2
    check(fg, n_gpu, got, lim_o, fl_o, n_o, margin, u)


def test_empty_queue_leaves_state_bitwise(K):
    """small higher modes and a large M: no cell is troubled and every cell
    clears the cheap positivity bound, so no block queues anything and the
    state is unchanged bit for bit"""
    k, nx, ny = 2, 67, 5
    u = W.random_euler_modes(np.random.default_rng(9), 9, nx * ny, amp=1e-4)
    om, s = setup(K, nx, ny, k, "euler", u)
    fg, n_gpu, got, lim_o, fl_o, n_o, margin = run_both(K, om, s, k, 1e12, u)
    assert n_gpu == 0 and n_o == 0
    assert not fg.any()
    assert np.array_equal(got, u)


@pytest.mark.parametrize("M", [0.0, 1500.0])
def test_scalar_limiter(K, M):
    """scalar advection (one component, no characteristic transform, no
    positivity test) through the same queue"""
    k, nx, ny = 2, 45, 13
    u = np.random.default_rng(11).standard_normal((1, 9, nx * ny))
    om, s = setup(K, nx, ny, k, "advection", u)
    fg, n_gpu, got, lim_o, fl_o, n_o, margin = run_both(K, om, s, k, M, u)
    assert np.any(fl_o & 1) and not np.any(fl_o & 6)
    check(fg, n_gpu, got, lim_o, fl_o, n_o, margin, u)
