"""The step under HIP graph capture.

Every call of the step path (crkdg_step_dev, crkdg_limit_dt) is a kernel
launch on the handle's stream: no host synchronisation, no allocation and no
memset, so a caller can capture a run of steps in a HIP graph and replay it.
The handle ping-pongs between two state buffers on the host side, so a
captured run holds an even number of steps (the host's buffer parity is the
same after it).  Checked: two steps (one-pass step, limiter, next dt) are
captured once and replayed four times, with eager work of another handle and
synchronisations between the replays; after every replay the state is
bitwise that of the same steps run eagerly, with the TVB test and with the
learned indicator (random parameters).
"""
import numpy as np
import pytest

from paper_2307_06471_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_06471_amd import crkdg
    return crkdg


def shock_solver(K, stream):
    import torch
    cfg = W.config("c5", scale=16)  # 256 x 64 cells
    params, xi = W.shock_problem(2000, cfg["nx"], cfg["ny"])
    x0, x1, y0, y1 = cfg["box"]
    mesh = K.make_mesh(2, cfg["nx"], cfg["ny"], x0=x0, x1=x1, y0=y0, y1=y1, bc=(2, 1, 1, 1),
                       bc_state=[W.post_shock_conserved(params[0])] * 4, equation=K.EQ_EULER,
                       gamma=W.GAMMA, precision=K.FP32_MIXED)
    s = K.Solver(mesh, cfg["k"], K.FLUX_LLF, 3, stream=stream)
    with torch.cuda.stream(stream):
        s.crkdg_project(K.IC_SHOCK, params, aux=torch.from_numpy(xi).cuda())
    s.crkdg_limit(50.0)
    return s, cfg


@pytest.mark.parametrize("indicator", ["tvb", "learned"])
def test_steps_replay_in_a_hip_graph(K, indicator):
    import torch
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    a, cfg = shock_solver(K, sa)   # eager
    b, _ = shock_solver(K, sb)     # captured
    assert a.crkdg_get_schedule() == K.SCHED_FUSED
    P = None
    lo = hi = 0.0
    if indicator == "learned":
        rng = np.random.default_rng(5)
        P = torch.from_numpy((0.3 * rng.standard_normal(1505)).astype(np.float32)).cuda()
        lo, hi = 0.3, 0.7
    flags_a = torch.zeros(a.ncells, dtype=torch.uint8, device="cuda")
    flags_b = torch.zeros(b.ncells, dtype=torch.uint8, device="cuda")
    dt_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_b = torch.zeros(1, dtype=torch.float64, device="cuda")
    a.crkdg_compute_dt(cfg["cfl"], dt_a)
    b.crkdg_compute_dt(cfg["cfl"], dt_b)
    torch.cuda.synchronize()

    def two_steps(s, dt, flags):
        for _ in range(2):
            s.crkdg_step_dev(dt)
            s.crkdg_limit_dt(50.0, cfg["cfl"], dt, flags, params=P, tau_lo=lo, tau_hi=hi)

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=sb):
        two_steps(b, dt_b, flags_b)
    torch.cuda.synchronize()
    # capture recorded the launches without running them
    assert np.array_equal(b.crkdg_get_state(), a.crkdg_get_state())
    for rep in range(4):
        with torch.cuda.stream(sa):
            two_steps(a, dt_a, flags_a)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ua, ub = a.crkdg_get_state(), b.crkdg_get_state()
        print(f"[graph] {indicator} replay {rep}: max |diff| {np.abs(ua - ub).max():.3e}, "
              f"dt {float(dt_a):.6e} / {float(dt_b):.6e}", flush=True)
        assert np.array_equal(ua, ub), rep
        assert float(dt_a) == float(dt_b)
        assert torch.equal(flags_a, flags_b)
