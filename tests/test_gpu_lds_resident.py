"""The LDS-resident solver for small 2D problems (one workgroup holds a whole
grid and runs every pass of every iteration): GD iterates (section II-B.1,
Eq. (2)) and spectral initialisation (section II-B.2, Eq. (3)-(4)) against
the FP64 oracle within 1e-4 after global-phase alignment, alone and running
beside the level launches of a larger problem in the same plan."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, make_plan, random_problem, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_IT = 1e-4


@pytest.fixture(autouse=True)
def lds_resident_on(monkeypatch):
    """The solver is opt-in; every test here runs with it switched on unless
    it says otherwise."""
    monkeypatch.setenv("SR_LDS_RESIDENT", "1")

# every supported axis length, radix-8-first (padded rows) and 3-factor rows,
# rectangular pads, ragged windows, L = 1..4, grids up to the LDS budget
SMALL = [
    ((24, 24), (64, 64), 2),
    ((12, 10), (16, 32), 1),
    ((40, 30), (96, 64), 3),
    ((100, 60), (128, 128), 2),
    ((70, 150), (96, 192), 1),
    ((120, 50), (256, 64), 4),
    ((9, 80), (16, 96), 2),
    ((30, 100), (32, 256), 3),
]
LARGE = ((200, 150), (512, 256), 2)  # runs as level launches beside them


def _plan_and_data(shapes, seed, dev, noisy_start=True):
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(seed)
    data = []
    for n_shape, m_shape, L in shapes:
        th, xs = random_problem(rng, n_shape, m_shape, L)
        op = oracle.StructuredOperator(th, n_shape)
        y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
        x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
        v0 = sr_inputs.complex_gaussian(rng, n_shape)
        eta = np.float32(oracle.default_step(op, y, 0.2))
        data.append(dict(th=th, op=op, y=y, x0=x0, v0=v0, eta=eta, n_shape=n_shape))
    plan = make_plan(shapes, [d["th"] for d in data], dev)
    srpr.sr_plan_set_schedule(plan, srpr.SR_SCHED_BATCHED)
    return plan, data


def _cat(arrs):
    return np.concatenate([np.asarray(a).ravel() for a in arrs])


@pytest.mark.parametrize("with_large", [False, True])
def test_lds_resident_gd(gpu, with_large):
    import torch
    import paper_2409_05734_amd as srpr
    shapes = SMALL + ([LARGE] if with_large else [])
    plan, data = _plan_and_data(shapes, 5 + with_large, gpu)
    y = to_dev(_cat([d["y"] for d in data]), gpu)
    eta = np.array([d["eta"] for d in data], np.float32)
    for k in (1, 7, 50):
        x = to_dev(_cat([d["x0"] for d in data]), gpu)
        srpr.sr_gd_solve(plan, y, x, k, eta)
        srpr.sr_plan_sync(plan)
        xh = to_host(x)
        for i, d in enumerate(data):
            xr = oracle.gd_solve(d["op"], d["y"], d["x0"], k, float(d["eta"]))
            xi = xh[plan.x_off[i]:plan.x_off[i + 1]].reshape(d["n_shape"])
            assert aligned(xi, xr) <= TOL_IT, (shapes[i], k)


@pytest.mark.parametrize("with_large", [False, True])
def test_lds_resident_spectral(gpu, with_large):
    import torch
    import paper_2409_05734_amd as srpr
    shapes = SMALL + ([LARGE] if with_large else [])
    plan, data = _plan_and_data(shapes, 9 + with_large, gpu)
    y = to_dev(_cat([d["y"] for d in data]), gpu)
    v0 = to_dev(_cat([d["v0"] for d in data]), gpu)
    for k in (0, 1, 10, 40):
        out = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
        srpr.sr_spectral_init(plan, y, v0, k, -1.0, out)
        srpr.sr_plan_sync(plan)
        xh = to_host(out)
        for i, d in enumerate(data):
            xr = oracle.spectral_init(d["op"], d["y"], d["v0"], k, -1.0)
            xi = xh[plan.x_off[i]:plan.x_off[i + 1]].reshape(d["n_shape"])
            assert rel_l2(xi, xr) <= TOL_IT, (shapes[i], k)


def test_lds_resident_is_deterministic(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    plan, data = _plan_and_data(SMALL[:3], 13, gpu)
    y = to_dev(_cat([d["y"] for d in data]), gpu)
    eta = np.array([d["eta"] for d in data], np.float32)
    outs = []
    for _ in range(2):
        x = to_dev(_cat([d["x0"] for d in data]), gpu)
        srpr.sr_gd_solve(plan, y, x, 30, eta)
        srpr.sr_plan_sync(plan)
        outs.append(x)
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("setting", [None, "1"])
def test_spectral_default_and_on(gpu, monkeypatch, setting):
    """Batched spectral solves run every problem on the level launches by
    default (unset switch) and the small ones in the LDS-resident solver with
    SR_LDS_RESIDENT=1; both against the oracle."""
    import torch
    import paper_2409_05734_amd as srpr
    if setting is None:
        monkeypatch.delenv("SR_LDS_RESIDENT", raising=False)
    else:
        monkeypatch.setenv("SR_LDS_RESIDENT", setting)
    shapes = SMALL[:4] + [LARGE]
    plan, data = _plan_and_data(shapes, 17, gpu)
    y = to_dev(_cat([d["y"] for d in data]), gpu)
    v0 = to_dev(_cat([d["v0"] for d in data]), gpu)
    out = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
    srpr.sr_spectral_init(plan, y, v0, 25, -1.0, out)
    srpr.sr_plan_sync(plan)
    xh = to_host(out)
    for i, d in enumerate(data):
        xr = oracle.spectral_init(d["op"], d["y"], d["v0"], 25, -1.0)
        xi = xh[plan.x_off[i]:plan.x_off[i + 1]].reshape(d["n_shape"])
        assert rel_l2(xi, xr) <= TOL_IT, (shapes[i], setting)
