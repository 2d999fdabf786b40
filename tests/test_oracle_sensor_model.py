"""Pins of the oracle's learned sensor model (per-pixel perceptron for the
measurement weight and truncation, §IV-B's "weight from the sensor's error
model") against facts that do not come from the oracle: exact bfloat16
rounding by rational arithmetic, closed-form features of planes, networks
whose arithmetic is exact (so a numpy product gives the answer), the reduction
of the zero network to constant weighting, a plane fused with per-pixel maps,
and finite differences of the binary64 loss."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2311_00626_amd import synth

NP = 2018
W1, B1, W2, B2, W3, B3 = 0, 864, 896, 1920, 1952, 2016


def bf16_exact(x: float) -> float:
    """Nearest bfloat16 (8 significant bits), ties to even, by rational arithmetic."""
    if x == 0 or not math.isfinite(x):
        return x
    f = Fraction(x)
    sign = -1 if f < 0 else 1
    f = abs(f)
    e = math.floor(math.log2(f))
    while Fraction(2) ** e > f:
        e -= 1
    while Fraction(2) ** (e + 1) <= f:
        e += 1
    q = Fraction(2) ** (e - 7)            # quantum of an 8-bit significand
    lo = (f // q) * q
    hi = lo + q
    if f - lo < hi - f:
        r = lo
    elif f - lo > hi - f:
        r = hi
    else:
        r = lo if (lo / q) % 2 == 0 else hi
    return float(sign * r)


def test_bf16_rounding_exact(oracle_mod):
    rng = np.random.default_rng(0)
    xs = (rng.standard_normal(3000) * 10.0 ** rng.uniform(-6, 6, 3000)).astype(np.float32)
    ties = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(2.0 + 2 ** -7), 0.75 + 2 ** -9]
    for x in list(xs) + [np.float32(t) for t in ties]:
        assert oracle_mod.round_bf16(float(x)) == bf16_exact(float(np.float32(x))), x


def plane_depth(cam, n_c, dist):
    """z-depth of the plane {p : n_c . p = dist} (camera frame) at pixel centres."""
    i = np.arange(cam.width) + 0.5
    j = np.arange(cam.height) + 0.5
    rx = (i[None, :] - cam.cx) / cam.fx
    ry = (j[:, None] - cam.cy) / cam.fy
    denom = n_c[0] * rx + n_c[1] * ry + n_c[2]
    return (dist / denom).astype(np.float32), rx, ry


@pytest.mark.parametrize("tilt_deg", [0.0, 35.0])
def test_features_of_a_plane(oracle_mod, tilt_deg):
    """Depth of a plane: the incidence angle is the angle between the pixel's
    ray and the plane normal (exact for a plane, whose central differences lie
    in it); the patch differences match the plane's depth differences."""
    cam = synth.PinholeCamera(40, 30, 35.0, 37.0, 19.0, 16.0)
    t = math.radians(tilt_deg)
    n_c = np.array([math.sin(t), 0.0, math.cos(t)])
    depth, rx, ry = plane_depth(cam, n_c, 2.0)
    feat = oracle_mod.sm_features(depth, cam.K, 5.0)
    ray = np.stack([rx + 0 * ry, ry + 0 * rx, np.ones_like(rx + ry)], -1)
    cosang = np.abs(ray @ n_c) / np.linalg.norm(ray, axis=-1)
    ang = np.arccos(np.clip(cosang, -1, 1))
    inner = (slice(1, -1), slice(1, -1))
    assert np.abs(feat[..., 26][inner] - ang[inner]).max() < 2e-4
    assert np.all(feat[0, :, 26] == np.float32(math.pi / 2)) and np.all(feat[:, -1, 26] == np.float32(math.pi / 2))
    assert np.array_equal(feat[..., 25], depth)
    # patch: entry (dj, di) = depth[j + dj, i + di] - depth[j, i] inside the image, else 0
    j, i = 12, 20
    for dj in range(-2, 3):
        for di in range(-2, 3):
            exp = np.float32(depth[j + dj, i + di] - depth[j, i])
            assert feat[j, i, (dj + 2) * 5 + di + 2] == np.clip(exp, -0.5, 0.5)
    assert np.all(feat[0, 0, :10] == 0.0)          # rows above the image
    assert feat[0, 0, 12] == 0.0                   # the centre


def test_features_step_edge_and_invalid(oracle_mod):
    cam = synth.PinholeCamera(16, 12, 14.0, 14.0, 8.0, 6.0)
    d = np.full((12, 16), 1.0, np.float32)
    d[:, 8:] = 3.0
    d[5, 5] = 0.0
    d[6, 10] = np.nan
    feat = oracle_mod.sm_features(d, cam.K, 5.0)
    assert feat[3, 7, 13] == 0.5 and feat[3, 8, 11] == -0.5          # clipped to +-0.5 m
    assert np.all(feat[5, 5] == 0.0) and np.all(feat[6, 10] == 0.0)   # invalid pixel: no features
    assert feat[5, 4, 13] == 0.0                                      # invalid neighbour: 0
    assert feat[4, 5, 26] == np.float32(math.pi / 2)                  # missing 4-neighbour


def exact_net(rng):
    """Sparse parameters with small dyadic values (drawn until every product,
    sum and activation of the forward is exact in bfloat16 and binary32)."""
    P = np.zeros(NP, np.float32)
    P[W1:B1] = rng.integers(-1, 2, 864) * (rng.random(864) < 0.15) * 0.25
    P[B1:W2] = rng.integers(0, 3, 32) * 0.25
    P[W2:B2] = rng.integers(-1, 2, 1024) * (rng.random(1024) < 0.15) * 0.5
    P[B2:W3] = rng.integers(0, 3, 32) * 0.25
    P[W3:B3] = rng.integers(-1, 2, 64) * 0.125
    P[B3:] = [0.5, -0.25]
    P[W1:B1].reshape(32, 27)[:, 26] = 0.0      # the angle feature is not dyadic
    return P


def exact_forward(P, x):
    Wm1 = P[W1:B1].reshape(32, 27).astype(np.float64)
    Wm2 = P[W2:B2].reshape(32, 32).astype(np.float64)
    Wm3 = P[W3:B3].reshape(2, 32).astype(np.float64)
    h1 = np.maximum(x @ Wm1.T + P[B1:W2], 0)
    h2 = np.maximum(h1 @ Wm2.T + P[B2:W3], 0)
    return h1, h2, h2 @ Wm3.T + P[B3:]


def test_forward_exact_network_equals_matrix_products(oracle_mod):
    """A network whose arithmetic is exact: the oracle's outputs equal the maps
    of numpy's matrix products (checks layout, biases, ReLU, output maps)."""
    rng = np.random.default_rng(1)
    cam = synth.PinholeCamera(8, 6, 7.0, 7.0, 4.0, 3.0)
    depth = (rng.integers(2, 7, (6, 8)) * 0.5).astype(np.float32)
    x = oracle_mod.sm_features(depth, cam.K, 5.0).astype(np.float64).reshape(-1, 27)
    x[:, 26] = 0.0
    for _ in range(50):
        P = exact_net(rng)
        h1, h2, o = exact_forward(P, x)
        vals = np.concatenate([x.reshape(-1), h1.reshape(-1), h2.reshape(-1)])
        if all(bf16_exact(float(v)) == v for v in vals) and np.all(np.abs(o) < 2 ** 20):
            break
    else:
        pytest.fail("no exact network drawn")
    assert (h1 > 0).mean() > 0.3 and np.count_nonzero(o) > 10
    w, e = oracle_mod.sm_maps(depth, cam.K, 5.0, 0.02, P)
    o0, o1 = o[:, 0], o[:, 1]
    w_exp = 0.5 * (o0 + np.sqrt(o0 * o0 + 4.0))
    s = 0.5 + 0.5 * (o1 / np.sqrt(1.0 + o1 * o1))
    e_exp = 0.02 * (1.0 + 7.0 * s)
    assert np.allclose(w.reshape(-1), w_exp, rtol=5e-7, atol=0)
    assert np.allclose(e.reshape(-1), e_exp, rtol=5e-7, atol=0)


def test_zero_network_is_constant_weighting(oracle_mod):
    """All-zero parameters: w = 1 and eps = 4.5 vs exactly, so learned fusion
    is bitwise the constant-weight fusion with truncation 4.5 voxels."""
    w_ = synth.box_room_sequence(0.05, n_frames=6)
    frames = w_.frames()
    P = np.zeros(NP, np.float32)
    vs = 0.05
    learned = oracle_mod.OracleMap(vs, 4.5, weighting="constant")
    const = oracle_mod.OracleMap(vs, 4.5, weighting="constant")
    for d, T in zip(frames, w_.poses):
        wm, em = oracle_mod.sm_maps(d, w_.camera.K, 5.0, vs, P)
        valid = (d > 0) & (d <= 5.0)
        assert np.all(wm[valid] == 1.0) and np.all(em[valid] == np.float32(4.5) * np.float32(vs))
        learned.integrate_learned(d, w_.camera.K, T, wm, em)
        const.integrate(d, w_.camera.K, T)
    a, b = learned.sorted_state(), const.sorted_state()
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_plane_with_per_pixel_maps(oracle_mod):
    """Fronto-parallel plane at Z0 with per-pixel weights and truncations: after
    one frame every voxel in front of its pixel's band has D = min(Z0 - z, eps_p)
    and W = w_p; none behind -eps_p is touched."""
    cam = synth.PinholeCamera(32, 24, 30.0, 30.0, 16.0, 12.0)
    Z0 = 1.5
    depth = np.full((24, 32), Z0, np.float32)
    rng = np.random.default_rng(2)
    wmap = rng.uniform(0.2, 3.0, (24, 32)).astype(np.float32)
    emap = rng.uniform(0.05, 0.3, (24, 32)).astype(np.float32)
    vs = 0.05
    m = oracle_mod.OracleMap(vs, 4.0, weighting="constant")
    m.integrate_learned(depth, cam.K, np.eye(4, dtype=np.float32), wmap, emap)
    blocks, dist, weight = m.sorted_state()
    g = (blocks[:, None, :] * 8 + np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8),
                                                       indexing="ij"), -1).reshape(-1, 3)[:, ::-1][None])
    # voxel order is lx + 8 ly + 64 lz
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    loc = np.stack([lx, ly, lz], -1).reshape(-1, 3)
    g = blocks[:, None, :] * 8 + loc[None]
    p = (g + 0.5) * np.float32(vs)
    z = p[..., 2]
    u = cam.fx * p[..., 0] / z + cam.cx
    v = cam.fy * p[..., 1] / z + cam.cy
    inside = (z > 0) & (u >= 0.01) & (u < 31.99) & (v >= 0.01) & (v < 23.99)
    frac_ok = (np.abs(u - np.round(u)) > 1e-3) & (np.abs(v - np.round(v)) > 1e-3)
    i = np.clip(u.astype(int), 0, 31)
    j = np.clip(v.astype(int), 0, 23)
    dp = Z0 - z
    ep, wp = emap[j, i], wmap[j, i]
    sel = inside & frac_ok & (dp > -ep + 1e-4)
    assert sel.sum() > 1000
    assert np.all(weight[sel] == wp[sel])
    assert np.abs(dist[sel] - np.minimum(dp[sel], ep[sel])).max() < 2e-6
    behind = inside & frac_ok & (dp < -ep - 1e-4)
    assert np.all(weight[behind] == 0)


def tiny_problem(seed=3):
    cam = synth.PinholeCamera(24, 18, 20.0, 20.0, 12.0, 9.0)
    room = synth.learning_room(1000, n_frames=30, camera=cam)
    clean, noisy = room.frames(count=30)
    idx = [0, 15, 29]
    frames = [noisy[k] for k in idx]
    poses = [room.poses[k] for k in idx]
    return cam, room, clean, frames, poses, idx


def loss_problem(oracle_mod, vs=0.1):
    cam, room, clean, frames, poses, idx = tiny_problem()
    params = synth.MapParams(vs, 4.0, "constant")
    om = oracle_mod.OracleMap.from_params(params, precision=64)
    for k in idx:
        om.integrate(clean[k], cam.K, room.poses[k])
    blocks, dist, weight = om.sorted_state()
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    loc = np.stack([lx, ly, lz], -1).reshape(-1, 3)
    g = (blocks[:, None, :] * 8 + loc[None]).reshape(-1, 3)
    D, W = dist.reshape(-1), weight.reshape(-1)
    keep = (W > 0) & (np.abs(D) < 4 * vs)
    return cam, frames, poses, g[keep].astype(np.int32), D[keep], vs


def test_loss_gradient_matches_finite_differences(oracle_mod):
    cam, frames, poses, vox, target, vs = loss_problem(oracle_mod)
    assert len(vox) > 200
    rng = np.random.default_rng(4)
    P = (rng.standard_normal(NP) * 0.05).astype(np.float32)
    P[B1:W2] = 0.1
    P[B2:W3] = 0.1
    loss, grad, used = oracle_mod.sm_loss_grad(P, frames, cam.K, poses, vs, 5.0, vox, target, emulate_bf16=False)
    assert used > 100 and loss > 0
    for trial in range(6):
        dirn = rng.standard_normal(NP)
        dirn /= np.linalg.norm(dirn)
        h = 2e-3
        lp = oracle_mod.sm_loss_grad((P + h * dirn).astype(np.float32), frames, cam.K, poses, vs, 5.0, vox,
                                     target, emulate_bf16=False)[0]
        lm = oracle_mod.sm_loss_grad((P - h * dirn).astype(np.float32), frames, cam.K, poses, vs, 5.0, vox,
                                     target, emulate_bf16=False)[0]
        # the perturbation actually applied is the binary32-rounded one
        dp = (P + h * dirn).astype(np.float32).astype(np.float64) - (P - h * dirn).astype(np.float32)
        fd = (lp - lm)
        an = float(grad @ dp)
        assert abs(fd - an) <= 2e-2 * abs(an) + 1e-9, (trial, fd, an)


def test_loss_is_zero_at_its_own_prediction(oracle_mod):
    """Targets equal to the model's own prediction: zero loss and gradient."""
    cam, frames, poses, vox, target, vs = loss_problem(oracle_mod)
    P = np.zeros(NP, np.float32)
    P[B3] = 0.5
    # prediction with these parameters = uncapped weighted average; w and eps are
    # constant (o = (0.5, 0)), so it is the constant-weight fusion at 4.5 voxels
    om = oracle_mod.OracleMap(vs, 4.5, precision=64, weighting="constant", max_weight=1e30)
    for d, T in zip(frames, poses):
        om.integrate(d, cam.K, T)
    blocks, dist, weight = om.sorted_state()
    lookup = {tuple(b): k for k, b in enumerate(blocks)}
    pred = np.array([dist[lookup[tuple(g // 8)], (g[0] % 8) + 8 * (g[1] % 8) + 64 * (g[2] % 8)]
                     if tuple(g // 8) in lookup else 0.0 for g in vox])
    loss, grad, used = oracle_mod.sm_loss_grad(P, frames, cam.K, poses, vs, 5.0, vox, pred, emulate_bf16=False)
    assert used > 100
    assert loss < 1e-24 and np.abs(grad).max() < 1e-12
