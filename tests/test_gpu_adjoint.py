"""GPU parity of the adjoint sweep (reverse streaming + transposed collision
Jacobian, checkpoint tape with segment recompute) against the oracle's
discrete adjoint, and of the torch.autograd.Function built on it."""

import numpy as np
import pytest

from tests.gpu_common import make_gpu, need_gpu, rel_l2, to_np, torch
from oracle import adjoint as oadj, run as orun
from paper_2001_11806_amd import inputs
from paper_2001_11806_amd.autograd import LBMFunction

pytestmark = pytest.mark.gpu

RATES = dict(omega=1 / 0.6, omega_bulk=1.0, omega_odd=0.0, magic=0.0, omega_hi=(1.0,) * 4)
METHOD_RATES = {"SRT": RATES, "TRT": dict(RATES, magic=3 / 16),
                "MRT": dict(RATES, omega_bulk=1.2, omega_hi=(1.3, 0.9, 1.1, 1.2))}


def _case(stencil="D3Q19", dims=(70, 10, 6), T=13, seed=4):
    nx, ny, nz = dims
    mask = inputs.channel_mask(nx, ny, nz)
    mask[2:4, 4:6, 30:33] = 1
    if stencil == "D2Q9":
        mask = mask[:1]
    u0 = inputs.uniform_noise_velocity(dims, 2e-2, seed, mask)
    if stencil == "D2Q9":
        u0[2] = 0
    rho = np.ones((nz, ny, nx))
    F = np.array([1e-3, 2e-4, 0.0 if stencil == "D2Q9" else -1e-4])
    return mask, rho, u0, F, T


def _gpu_gradient(stencil, dtype, dims, mask, rho, u0, F, T, k, pattern=0, method="SRT"):
    g = make_gpu(stencil, method, dtype, dims, mask, METHOD_RATES[method], checkpoint_every=k, max_tape_steps=T,
                 pattern=pattern)
    g.set_force(F)
    g.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
    g.step(T)
    # loss gradient at the GPU's own final state, as the oracle would seed it
    _, u_T = g.macroscopic()
    dL_du = torch.zeros_like(u_T)
    fl = torch.tensor(mask == 0, device=u_T.device)
    dL_du[0, :, :, -1] = 2 * u_T[0, :, :, -1] * fl[:, :, -1]
    g.adjoint_seed(dL_du)
    g.adjoint_step(T)
    du, drho, dF = g.adjoint_grads(want_rho=True)
    g.close()
    return to_np(du), to_np(drho), dF


@pytest.mark.parametrize("method", ["SRT", "TRT", "MRT"])
@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("k", [1, 4, 13])
def test_adjoint_fp64_matches_oracle(stencil, k, method):
    need_gpu()
    dims = (70, 10, 1) if stencil == "D2Q9" else (70, 10, 6)
    mask, rho, u0, F, T = _case(stencil, dims)
    print("case", stencil, method, "k", k, flush=True)
    du, drho, dF = _gpu_gradient(stencil, "f64", dims, mask, rho, u0, F, T, k, method=method)
    cfg = orun.Config(stencil, method, METHOD_RATES[method])
    L, gu, grho, gF = oadj.gradient(cfg, rho, u0, mask, F, T)
    assert rel_l2(du, gu) <= 1e-10
    assert rel_l2(drho, grho) <= 1e-10
    np.testing.assert_allclose(dF, gF, rtol=1e-10)


@pytest.mark.parametrize("method", ["SRT", "TRT", "MRT"])
def test_adjoint_fp32_matches_oracle(method):
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, T = _case("D3Q19", dims)
    du, drho, dF = _gpu_gradient("D3Q19", "f32", dims, mask, rho, u0, F, T, 5, method=method)
    cfg = orun.Config("D3Q19", method, METHOD_RATES[method])
    L, gu, grho, gF = oadj.gradient(cfg, rho, u0, mask, F, T)
    e_u, e_F = rel_l2(du, gu), rel_l2(dF, gF)
    print("fp32 adjoint: rel L2 dL/du0 %.2e, dL/dF %.2e" % (e_u, e_F))
    assert e_u <= 1e-4 and e_F <= 1e-4


def test_autograd_function_matches_oracle():
    """LBMFunction: torch loss on u_T, backward through the adjoint sweep."""
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, T = _case("D3Q19", dims)
    lbm = make_gpu("D3Q19", "SRT", "f64", dims, mask, RATES, checkpoint_every=5, max_tape_steps=T)
    u0_t = torch.tensor(u0, device="cuda", requires_grad=True)
    F_t = torch.tensor(F, device="cuda", requires_grad=True)
    u_T = LBMFunction.apply(u0_t, F_t, lbm, T, torch.tensor(rho, device="cuda"))
    fl = torch.tensor(mask == 0, device="cuda")
    loss = ((u_T[0, :, :, -1] * fl[:, :, -1]) ** 2).sum()
    loss.backward()
    cfg = orun.Config("D3Q19", "SRT", RATES)
    L, gu, grho, gF = oadj.gradient(cfg, rho, u0, mask, F, T)
    assert abs(loss.item() / L - 1) < 1e-12
    assert rel_l2(to_np(u0_t.grad), gu) <= 1e-10
    np.testing.assert_allclose(to_np(F_t.grad), gF, rtol=1e-10)
    lbm.close()


def test_adjoint_state_errors():
    need_gpu()
    from paper_2001_11806_amd.lbm import LBMError
    dims = (64, 6, 4)
    g = make_gpu("D3Q19", "SRT", "f32", dims, None, RATES, checkpoint_every=4, max_tape_steps=8)
    g.init_equilibrium()
    g.step(9)
    with pytest.raises(LBMError, match="max_tape_steps"):
        g.adjoint_seed(torch.zeros(3, 4, 6, 64, device="cuda"))
    g.init_equilibrium()
    g.step(8)
    g.adjoint_seed(torch.zeros(3, 4, 6, 64, device="cuda"))
    with pytest.raises(LBMError, match="remain"):
        g.adjoint_step(9)
    with pytest.raises(LBMError, match="t = 0"):
        g.adjoint_grads()
    with pytest.raises(LBMError, match="LBM_ESTATE.*initial fields"):
        g.set_pdfs(torch.zeros(19, 4, 6, 64, dtype=torch.float64, device="cuda"))
    g.close()


def test_adjoint_with_moving_wall_matches_oracle():
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, T = _case("D3Q19", dims)
    mask = mask.copy()
    mask[:, -1, :] = 2
    u0 = u0 * (mask == 0)
    table = np.zeros((3, 3))
    table[2] = (0.03, 0.0, 0.01)
    g = make_gpu("D3Q19", "SRT", "f64", dims, mask, RATES, checkpoint_every=4, max_tape_steps=T)
    g.set_force(F)
    g.set_wall_velocity(2, table[2])
    g.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
    g.step(T)
    _, u_T = g.macroscopic()
    dL = torch.zeros_like(u_T)
    fl = torch.tensor(mask == 0, device=u_T.device)
    dL[0, :, :, -1] = 2 * u_T[0, :, :, -1] * fl[:, :, -1]
    g.adjoint_seed(dL)
    g.adjoint_step(T)
    du, _, dF = g.adjoint_grads()
    g.close()
    cfg = orun.Config("D3Q19", "SRT", RATES)
    L, gu, grho, gF = oadj.gradient(cfg, rho, u0, mask, F, T, wall_velocity=table)
    assert rel_l2(to_np(du), gu) <= 1e-10
    np.testing.assert_allclose(dF, gF, rtol=1e-10)


@pytest.mark.parametrize("method", ["SRT", "TRT", "MRT"])
@pytest.mark.parametrize("stencil", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
@pytest.mark.parametrize("T,k", [(13, 4), (12, 5), (7, 1)])
def test_aa_adjoint_equals_two_arrays(stencil, dtype, T, k, method):
    """AA pattern with a tape: the checkpoints are stored in the two-array
    layout and lambda is updated in place by the transposed AA kernels.  The
    recomputed states and every per-cell transpose are the two-array ones, so
    all gradients agree bit for bit, for odd and even T."""
    need_gpu()
    dims = (70, 10, 1) if stencil == "D2Q9" else (70, 10, 6)
    mask, rho, u0, F, _ = _case(stencil, dims)
    print("case AA adjoint", stencil, method, dtype, "T", T, "k", k, flush=True)
    a = _gpu_gradient(stencil, dtype, dims, mask, rho, u0, F, T, k, pattern=0, method=method)
    b = _gpu_gradient(stencil, dtype, dims, mask, rho, u0, F, T, k, pattern=1, method=method)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(np.asarray(a[2]), np.asarray(b[2]))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_aa_adjoint_matches_oracle_with_moving_wall(dtype):
    """AA adjoint with a moving wall: equal bit for bit to the two-array
    adjoint (the AA slots hold post-collision values, so the initial
    checkpoint relaid out of the AA layout is an exact copy), and in FP64
    against the oracle."""
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, T = _case("D3Q19", dims)
    mask = mask.copy()
    mask[:, -1, :] = 2
    u0 = u0 * (mask == 0)
    table = np.zeros((3, 3))
    table[2] = (0.03, 0.0, 0.01)
    grads = []
    for pattern in (0, 1):
        g = make_gpu("D3Q19", "SRT", dtype, dims, mask, RATES, checkpoint_every=3, max_tape_steps=T,
                     pattern=pattern)
        g.set_force(F)
        g.set_wall_velocity(2, table[2])
        g.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
        g.step(T)
        _, u_T = g.macroscopic()
        dL = torch.zeros_like(u_T)
        fl = torch.tensor(mask == 0, device=u_T.device)
        dL[0, :, :, -1] = 2 * u_T[0, :, :, -1] * fl[:, :, -1]
        g.adjoint_seed(dL)
        g.adjoint_step(T)
        grads.append(g.adjoint_grads(want_rho=True))
        g.close()
    (du, drho, dF), (du1, drho1, dF1) = grads
    assert torch.equal(du, du1) and torch.equal(drho, drho1)
    assert np.array_equal(np.asarray(dF), np.asarray(dF1))
    if dtype == "f64":
        cfg = orun.Config("D3Q19", "SRT", RATES)
        L, gu, grho, gF = oadj.gradient(cfg, rho, u0, mask, F, T, wall_velocity=table)
        assert rel_l2(to_np(du), gu) <= 1e-10
        assert rel_l2(to_np(drho), grho) <= 1e-10
        np.testing.assert_allclose(dF, gF, rtol=1e-10)


def test_autograd_function_aa_pattern():
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, T = _case("D3Q19", dims)
    lbm = make_gpu("D3Q19", "SRT", "f64", dims, mask, RATES, checkpoint_every=5, max_tape_steps=T, pattern=1)
    u0_t = torch.tensor(u0, device="cuda", requires_grad=True)
    F_t = torch.tensor(F, device="cuda", requires_grad=True)
    u_T = LBMFunction.apply(u0_t, F_t, lbm, T, torch.tensor(rho, device="cuda"))
    fl = torch.tensor(mask == 0, device="cuda")
    loss = ((u_T[0, :, :, -1] * fl[:, :, -1]) ** 2).sum()
    loss.backward()
    cfg = orun.Config("D3Q19", "SRT", RATES)
    L, gu, grho, gF = oadj.gradient(cfg, rho, u0, mask, F, T)
    assert abs(loss.item() / L - 1) < 1e-12
    assert rel_l2(to_np(u0_t.grad), gu) <= 1e-10
    np.testing.assert_allclose(to_np(F_t.grad), gF, rtol=1e-10)
    lbm.close()


@pytest.mark.parametrize("pattern", [0, 1])
@pytest.mark.parametrize("method", ["SRT", "MRT"])
def test_adjoint_in_xcd_slab_order_matches_oracle(method, pattern):
    """48 rows: the forward, recompute and adjoint launches use the XCD-slab
    block order with alternating directions; the gradients keep the FP64 bar."""
    need_gpu()
    dims = (70, 8, 6)
    mask, rho, u0, F, T = _case("D3Q19", dims)
    du, drho, dF = _gpu_gradient("D3Q19", "f64", dims, mask, rho, u0, F, T, 4, pattern=pattern, method=method)
    cfg = orun.Config("D3Q19", method, METHOD_RATES[method])
    L, gu, grho, gF = oadj.gradient(cfg, rho, u0, mask, F, T)
    assert rel_l2(du, gu) <= 1e-10
    assert rel_l2(drho, grho) <= 1e-10
    np.testing.assert_allclose(dF, gF, rtol=1e-10)


def _tape_ctx(dims, mask, k, T, pattern=0, dtype="f64"):
    g = make_gpu("D3Q19", "SRT", dtype, dims, mask, RATES, checkpoint_every=k, max_tape_steps=T, pattern=pattern)
    return g


def _seeded_grads(g, mask):
    _, u_T = g.macroscopic()
    dL = torch.zeros_like(u_T)
    fl = torch.tensor(mask == 0, device=u_T.device)
    dL[0, :, :, -1] = 2 * u_T[0, :, :, -1] * fl[:, :, -1]
    g.adjoint_seed(dL)
    g.adjoint_step(g.time)
    return g.adjoint_grads(want_rho=True)


@pytest.mark.parametrize("pattern", [0, 1])
def test_state_survives_the_adjoint_and_the_forward_continues(pattern):
    """With a tape the two-array sweep writes each checkpoint straight into
    its tape slot, so the current state may live there (T = 16) or in a grid
    (T = 13); the adjoint must not disturb it: readout and PDFs are unchanged
    after a full adjoint pass, and further steps match a run without a tape
    bit for bit, solid cells included (they are kept in the grids only)."""
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, _ = _case("D3Q19", dims)
    ref = make_gpu("D3Q19", "SRT", "f64", dims, mask, RATES, pattern=pattern)
    ref.set_force(F)
    ref.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
    g = _tape_ctx(dims, mask, 4, 40, pattern)
    g.set_force(F)
    g.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
    for T in (13, 16):   # the state in a grid, then in a tape slot
        g.step(T - g.time)
        ref.step(T - ref.time)
        before = g.get_pdfs()
        assert torch.equal(before, ref.get_pdfs()), T
        _seeded_grads(g, mask)
        assert torch.equal(g.get_pdfs(), before), T
        (ra, ua), (rb, ub) = g.macroscopic(), ref.macroscopic()
        assert torch.equal(ua, ub) and torch.equal(ra, rb), T
    g.step(7)
    ref.step(7)
    assert torch.equal(g.get_pdfs(), ref.get_pdfs())
    g.close()
    ref.close()


def test_seed_again_after_continuing_within_a_segment():
    """T = 13, adjoint, two more steps (still in the same segment of k = 4),
    seed again: the second pass recomputes from the same tape and its
    gradients equal those of a fresh 15-step run bit for bit."""
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, _ = _case("D3Q19", dims)
    a = _tape_ctx(dims, mask, 4, 20)
    a.set_force(F)
    a.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
    a.step(13)
    _seeded_grads(a, mask)
    a.step(2)
    ga = _seeded_grads(a, mask)
    b = _tape_ctx(dims, mask, 4, 20)
    b.set_force(F)
    b.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
    b.step(15)
    gb = _seeded_grads(b, mask)
    assert torch.equal(ga[0], gb[0]) and torch.equal(ga[1], gb[1])
    assert np.array_equal(np.asarray(ga[2]), np.asarray(gb[2]))
    a.close()
    b.close()


@pytest.mark.parametrize("pattern", [0, 1])
@pytest.mark.parametrize("T", [20, 18, 17, 16])
def test_last_segment_kept_from_the_forward(pattern, T):
    """max_tape_steps = 20, k = 4: the forward keeps the states 17..19 of the
    last segment in the segment buffer, so an adjoint seeded at T = 17 ... 20
    skips that recompute (at T < 20 the current state lives there and moves
    to a grid first).  Gradients and the state itself equal those of a
    context whose tape reaches further (max_tape_steps = 40, where T is not
    in the last segment and everything is recomputed), bit for bit."""
    need_gpu()
    dims = (70, 10, 6)
    mask, rho, u0, F, _ = _case("D3Q19", dims)
    out = []
    for max_T in (20, 40):
        g = _tape_ctx(dims, mask, 4, max_T, pattern)
        g.set_force(F)
        g.init_equilibrium(torch.tensor(rho), torch.tensor(u0))
        g.step(T)
        before = g.get_pdfs()
        grads = _seeded_grads(g, mask)
        assert torch.equal(g.get_pdfs(), before)
        g.step(2 if max_T == 40 or T <= 18 else 0)
        out.append((grads, before, g.get_pdfs()))
        g.close()
    (ga, pa, qa), (gb, pb, qb) = out
    assert torch.equal(pa, pb)
    assert torch.equal(ga[0], gb[0]) and torch.equal(ga[1], gb[1])
    assert np.array_equal(np.asarray(ga[2]), np.asarray(gb[2]))
    if T <= 18:
        assert torch.equal(qa, qb)
