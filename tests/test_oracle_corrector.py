"""Pins of the corrector network and features (FP64 oracle): backpropagation
against central finite differences, closed forms of special weights, the
first Adam step, rigid-body fields (zero features, exact labels), interface
cell counts by lattice-point counting, and the feature ordering."""
import math

import numpy as np

import synth
from oracle import corrector as oc
from oracle import mlp, stats


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    theta = synth.mlp_initial_params(3) + rng.normal(0, 0.05, mlp.N_PARAMS)
    X = rng.normal(size=(7, 85))
    T = rng.normal(size=(7, 9))
    L, g = mlp.grad(theta, X, T)
    assert math.isclose(L, mlp.loss(theta, X, T), rel_tol=1e-14)
    idx = rng.choice(mlp.N_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, [0, 5439, 5440 + 63, 5504, 9663, 9664, 10239, 10240, 10248]])
    h = 1e-6
    fd = np.empty(len(idx))
    for n, i in enumerate(idx):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[n] = (mlp.loss(tp, X, T) - mlp.loss(tm, X, T)) / (2 * h)
    assert np.linalg.norm(g[idx] - fd) <= 1e-6 * np.linalg.norm(fd)


def test_mlp_special_weights():
    X = np.random.default_rng(1).normal(size=(5, 85))
    theta = np.zeros(mlp.N_PARAMS)
    theta[-9:] = np.arange(9) * 0.1 - 0.3
    y, _ = mlp.forward(theta, X)
    assert np.array_equal(y, np.broadcast_to(theta[-9:], (5, 9)))
    # one path: input 5 -> hidden 0 -> hidden 0 -> output 2 ([out][in] weights)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(np.zeros(mlp.N_PARAMS))
    W1[0, 5], b1[0], W2[0, 0], b2[0], W3[2, 0], b3[2] = 1.7, 0.1, -0.8, 0.05, 1.3, 0.2
    y, _ = mlp.forward(mlp.pack([W1, b1, W2, b2, W3, b3]), X)

    def silu(z):
        return z / (1.0 + math.exp(-z))

    for b in range(5):
        h1 = silu(1.7 * X[b, 5] + 0.1)
        want = 1.3 * silu(-0.8 * h1 + 0.05) + 0.2
        assert math.isclose(y[b, 2], want, rel_tol=1e-13)
        assert y[b, 0] == 0.0
    z = np.linspace(-6, 6, 25)
    assert np.allclose(mlp.silu_grad(z), (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6, rtol=1e-8, atol=1e-10)
    assert mlp.silu(np.array([0.0]))[0] == 0.0 and abs(mlp.silu(np.array([40.0]))[0] - 40.0) < 1e-12


def test_adam_first_step_and_descent():
    rng = np.random.default_rng(2)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(t1 - theta, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a few hundred steps fit a smooth target
    X = rng.normal(size=(64, 85))
    T = np.tanh(X[:, :9] * 0.5)
    th = synth.mlp_initial_params(0)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = mlp.loss(th, X, T)
    for t in range(1, 301):
        _, gg = mlp.grad(th, X, T)
        th, m, v = mlp.adam_step(th, gg, m, v, t, lr=3e-3)
    assert mlp.loss(th, X, T) < 0.05 * L0


def _rigid_field(shape, Xc, U, Om):
    xyz = stats.node_coords(shape)
    d = np.stack([xyz[k] - Xc[k] for k in range(3)])
    return U[:, None, None, None] + np.cross(Om, d, axis=0)


def test_rigid_rotation_gives_zero_features_and_exact_labels():
    """A field that is one rigid-body motion everywhere: relative velocities
    vanish, the masked field is that motion, central differences are exact
    (the field is linear; the sphere sits away from the periodic seam), so
    the labels equal the rotation tensor / u_rms and the dissipation is 0."""
    shape = (40, 40, 40)
    Xc = np.array([19.6, 20.3, 20.1])
    U = np.array([0.01, -0.004, 0.002])
    Om = np.array([0.0008, -0.0011, 0.0005])
    u = _rigid_field(shape, Xc, U, Om)
    X, r, rd = Xc[None], np.array([6.0]), 0.4
    flat, part = oc.interface_cells(shape, X, r, rd, 0.0, 10.0)
    assert len(flat) > 500 and np.all(part == 0)
    F = oc.features(u, flat, part, X, U[None], Om[None], r, 0.03, shape)
    assert np.abs(F[:, :81]).max() < 1e-15
    xyz = oc._node_xyz(flat, shape)
    dist = np.linalg.norm(xyz - Xc, axis=1)
    assert np.allclose(F[:, 81], dist - 6.0, rtol=0, atol=1e-13)
    assert np.allclose(np.linalg.norm(F[:, 82:85], axis=1), 1.0, atol=1e-14)
    assert (F[:, 81] >= 0).all() and (F[:, 81] < 2 - rd).all()
    owner, _ = stats.classify(shape, X, r)
    T = oc.labels(u, owner, X, U[None], Om[None], flat, 0.03, shape)
    A = np.array([[0, -Om[2], Om[1]], [Om[2], 0, -Om[0]], [-Om[1], Om[0], 0]])
    assert np.allclose(T, np.broadcast_to(A.ravel() / 0.03, T.shape), rtol=0, atol=1e-13)
    assert np.abs(oc.dissipation_from_gradient(T * 0.03, 0.01)).max() < 1e-25
    # identical paired fields: zero targets; a zero correction leaves G_plain
    assert np.abs(oc.targets(T, T)).max() == 0.0
    assert np.array_equal(oc.corrected_gradient(T, np.zeros_like(T), 0.03), T * 0.03)


def _count_in_sphere(X, R, shape):
    nx, ny, nz = shape
    n = 0
    for z in range(nz):
        dz = min((z - X[2]) % nz, (X[2] - z) % nz)
        for y in range(ny):
            dy = min((y - X[1]) % ny, (X[1] - y) % ny)
            rem = R * R - dy * dy - dz * dz
            if rem <= 0:
                continue
            h = math.sqrt(rem)
            lo, hi = math.floor(X[0] - h) + 1, math.ceil(X[0] + h) - 1
            n += max(0, hi - lo + 1)
    return n


def test_interface_cell_counts_and_fallback():
    shape = (56, 40, 40)
    rd = 0.4
    X = np.array([[12.3, 20.2, 19.7], [27.9, 20.6, 20.4], [44.0, 12.0, 30.0]])
    r = np.array([6.0, 5.0, 5.5])
    # the isolated sphere keeps its whole band: count by lattice points
    flat, part = oc.interface_cells(shape, X[2:], r[2:], rd, 0.0, 10.0)
    want = _count_in_sphere(X[2], r[2] - rd + 2, shape) - _count_in_sphere(X[2], r[2], shape)
    assert len(flat) == want
    # with the close pair present, check every candidate by brute force
    flat, part = oc.interface_cells(shape, X, r, rd, 0.0, 10.0)
    nx, ny, _ = shape
    L = np.array(shape, float)
    got = dict(zip(flat.tolist(), part.tolist()))
    n_ok = 0
    for p in range(3):
        lo = np.floor(X[p] - 8).astype(int)
        for z in range(lo[2], lo[2] + 17):
            for y in range(lo[1], lo[1] + 17):
                for x in range(lo[0], lo[0] + 17):
                    node = np.array([x % shape[0], y % shape[1], z % shape[2]], float)
                    dd = [np.linalg.norm((node - X[q] + L / 2) % L - L / 2) for q in range(3)]
                    inband = r[p] <= dd[p] < r[p] - rd + 2
                    clear = all(dd[q] >= r[q] - rd + 2 + math.sqrt(3) for q in range(3) if q != p)
                    key = int(node[0] + nx * (node[1] + ny * node[2]))
                    if inband and clear:
                        assert got.get(key) == p
                        n_ok += 1
                    elif inband:
                        assert key not in got
    assert n_ok == len(flat)
    # the training range selects d exactly
    flat2, _ = oc.interface_cells(shape, X, r, rd, 0.5, 1.0)
    F = oc.features(np.zeros((3,) + shape[::-1]), flat, part, X, np.zeros((3, 3)), np.zeros((3, 3)), r, 1.0, shape)
    sel = (F[:, 81] >= 0.5) & (F[:, 81] <= 1.0)
    assert np.array_equal(np.sort(flat2), np.sort(flat[sel]))


def test_feature_ordering_and_relative_velocity():
    """u_x = f(z) only: stencil entry o = 9 (oz + 1) + 3 (oy + 1) + (ox + 1);
    (0, 0, +1) is o = 22, so feature 66 is (f(z + 1) - U_x) / u_rms."""
    shape = (30, 30, 30)
    zz = np.arange(30, dtype=float)
    f = 0.01 * np.sin(0.3 * zz) + 0.002 * zz
    u = np.zeros((3, 30, 30, 30))
    u[0] = f[:, None, None]
    X = np.array([[15.2, 14.8, 15.1]])
    U = np.array([[0.003, 0.0, 0.0]])
    flat, part = oc.interface_cells(shape, X, np.array([5.0]), 0.0, 0.0, 10.0)
    F = oc.features(u, flat, part, X, U, np.zeros((1, 3)), np.array([5.0]), 0.02, shape)
    z = flat // 900
    assert np.allclose(F[:, 66], (f[(z + 1) % 30] - 0.003) / 0.02, rtol=0, atol=1e-14)
    assert np.allclose(F[:, 39], (f[z] - 0.003) / 0.02, rtol=0, atol=1e-14)       # centre, o = 13
    assert np.allclose(F[:, 12], (f[(z - 1) % 30] - 0.003) / 0.02, rtol=0, atol=1e-14)  # o = 4: oz = -1
    assert np.allclose(F[:, 0], (f[(z - 1) % 30] - 0.003) / 0.02, rtol=0, atol=1e-14)   # o = 0: all -1
    assert np.abs(F[:, 1:81:3]).max() == 0.0 and np.abs(F[:, 2:81:3]).max() == 0.0


def test_corrected_statistics_replace_only_the_cells():
    shape = (24, 24, 24)
    rng = np.random.default_rng(5)
    u = rng.normal(size=(3, 24, 24, 24)) * 0.01
    X = np.array([[12.0, 12.0, 12.0]])
    r = np.array([5.0])
    flat, part = oc.interface_cells(shape, X, r, 0.4, 0.0, 10.0)
    G = rng.normal(size=(len(flat), 9)) * 1e-3
    s0 = stats.statistics(u, np.ones(u.shape[1:]), 0.01, shape, X, None, None, r, nbins=16)
    s1 = stats.statistics(u, np.ones(u.shape[1:]), 0.01, shape, X, None, None, r, nbins=16, corrected=(flat, G))
    assert s0["eps_fluid_corrected"] == s0["eps_fluid"] and s0["n_corrected"] == 0
    assert np.array_equal(s0["hist"][5], s0["hist"][2])
    owner, _ = stats.classify(shape, X, r)
    um = stats.masked_velocity(u, owner, X, np.zeros((1, 3)), np.zeros((1, 3)), shape)
    eps = stats.dissipation_field(um, 0.01).ravel()
    delta = oc.dissipation_from_gradient(G, 0.01).sum() - eps[flat].sum()
    assert math.isclose(s1["eps_fluid_corrected"] * s1["n_fluid"], s0["eps_fluid"] * s0["n_fluid"] + delta,
                        rel_tol=1e-12)
    assert s1["n_corrected"] == len(flat) and np.array_equal(s1["hist"][2], s0["hist"][2])
