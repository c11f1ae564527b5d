"""Pins of the oracle's permutohedral-lattice filter and mean-field update
(the message passing of the continuous CRF, Sec. 3.5.3).

* Simplex: the d+1 vertices lie on the lattice (coordinates sum to zero,
  all congruent mod d+1 after the canonical shift), the barycentric weights
  are in [0,1] and sum to 1, and the weighted vertices reproduce the lifted
  position (lifting written here from the definition of the lattice scale).
* Splat / blur / slice against the same steps written with a Python dict
  over full lattice coordinates, the blur directions taken from the lattice
  definition; d = 1 against linear splatting, two [1,2,1]/4 passes and
  linear slicing on the integer line (numpy); far clusters do not interact.
* Mean field: zero pairwise weight gives softmax(-unary); with a Potts
  weight, the update equals softmax(-unary + w F(Q)) computed here from the
  oracle's own filter (one step), and distributions stay normalised.
* Mean field with a compatibility matrix mu: mu = 0 gives softmax(-unary);
  the textbook Potts matrix w (1 - I) gives the Potts result above (the
  per-point constant w sum_l F_l cancels in the softmax); an asymmetric mu
  on one isolated point (its filter is a scalar multiple c of Q, c the
  filter of ones) against the two-label closed form, which a transposed mu
  fails.
* Filter adjoint: <F x, y> = <x, F^T y> for random x, y, d = 1, 3, 6.
* Width and isotropy of the Gaussian (Eq. 20's kernel with unit standard
  deviation per scaled feature axis), d = 2, 3, 4, 6, derived from the
  lattice's geometry and not from the lift's per-axis factors: on a dense
  uniform point cloud the normalised moments F(s)/F(1) and F(s^2)/F(1) of
  the coordinate s = u.x along the axes and random unit directions u give a
  mean at the point and a variance of 1 in every direction; the response
  to ones integrates to the density times the feature-space volume per
  lattice vertex.
* Mean-field gradient (learning the compatibility matrix): the gradients
  with respect to mu and to the unaries against central differences of
  <gQ, Q_T> through the oracle's forward.
"""
import numpy as np
import pytest


def _lift(p):
    """Position on the plane sum x = 0 of R^{d+1}, lattice scale of the method."""
    N, d = p.shape
    el = np.zeros((N, d + 1))
    sm = np.zeros(N)
    for i in range(d, 0, -1):
        scale = (d + 1) * np.sqrt(2.0 / 3.0) / np.sqrt(i * (i + 1))
        cf = p[:, i - 1] * scale
        el[:, i] = sm - i * cf
        sm += cf
    el[:, 0] = sm
    return el


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 22])
def test_simplex_reproduces_the_lifted_position(oracle_lib, d):
    rng = np.random.default_rng(d)
    p = rng.normal(scale=3.0, size=(500, d)).astype(np.float32)
    keys, w = oracle_lib.lattice_simplex(p)
    full = np.concatenate([keys, -keys.sum(-1, keepdims=True)], -1).astype(np.float64)  # [N,d+1,d+1]
    # every vertex: coordinates congruent to each other mod d+1 (a lattice point)
    m = np.mod(full, d + 1)
    assert (m == m[..., :1]).all()
    assert (w >= -1e-6).all() and (w <= 1 + 1e-6).all()
    np.testing.assert_allclose(w.sum(-1), 1.0, atol=1e-9)
    rec = (w[..., None] * full).sum(1)
    np.testing.assert_allclose(rec, _lift(p.astype(np.float64)), atol=2e-5 * (1 + np.abs(p).max()))
    # Independently of the lift's per-axis factors: the lift is (d+1) sqrt(2/3)
    # times an isometry onto the plane sum x = 0, so the reconstructed points
    # keep every inner product up to that factor (a wrong factor on any axis
    # i breaks it for the points' i-th components).
    P = p.astype(np.float64)
    np.testing.assert_allclose(rec.sum(-1), 0.0, atol=1e-4 * (1 + np.abs(rec).max()))
    gram = rec @ rec.T
    want = (2.0 / 3.0) * (d + 1) ** 2 * (P @ P.T)
    assert np.abs(gram - want).max() <= 1e-5 * np.abs(want).max() * (d + 1), d
    # the d+1 vertices are distinct and pairwise adjacent (differ by a 0/1 pattern times d+1 shift)
    for i in range(0, 500, 50):
        assert len({tuple(v) for v in keys[i]}) == d + 1


def _dict_filter(keys, w, v):
    """Splat / blur / slice written with a Python dict over full lattice
    coordinates (d+1 of them, summing to zero); blur direction j moves by
    +-((1,...,1) - (d+1) e_j), vertices that were never splatted stay absent."""
    N, d1, d = keys.shape
    full = np.concatenate([keys, -keys.sum(-1, keepdims=True)], -1)
    lat = {}
    for i in range(N):
        for r in range(d1):
            k = tuple(full[i, r])
            lat[k] = lat.get(k, 0.0) + w[i, r] * v[i]
    for j in range(d1):
        step = np.ones(d1, int)
        step[j] -= d1
        new = {}
        for k, val in lat.items():
            kk = np.array(k)
            acc = 0.5 * val
            for sgn in (-1, 1):
                nb = tuple(kk + sgn * step)
                if nb in lat:
                    acc = acc + 0.25 * lat[nb]
            new[k] = acc
        lat = new
    out = np.zeros_like(v)
    for i in range(N):
        for r in range(d1):
            out[i] += w[i, r] * lat[tuple(full[i, r])]
    return out, len(lat)


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_filter_matches_dict_lattice(oracle_lib, d):
    rng = np.random.default_rng(20 + d)
    p = rng.normal(scale=1.5, size=(250, d)).astype(np.float32)
    v = rng.normal(size=(250, 2))
    out, nv = oracle_lib.lattice_filter(p, v)
    keys, w = oracle_lib.lattice_simplex(p)
    want, n_want = _dict_filter(keys, w, v)
    np.testing.assert_allclose(out, want, rtol=1e-10, atol=1e-12)
    assert nv == n_want


def test_d1_filter_is_linear_splat_blur_slice(oracle_lib):
    """d = 1: the lattice is the integer line (coordinate 2/sqrt(3) p); the
    filter is linear splatting, two [1,2,1]/4 passes over the splatted
    points, and linear slicing."""
    rng = np.random.default_rng(7)
    p = rng.uniform(-2.0, 2.0, size=(400, 1)).astype(np.float32)
    v = rng.normal(size=(400, 2))
    out, nv = oracle_lib.lattice_filter(p, v)
    y = p[:, 0].astype(np.float64) * 2.0 / np.sqrt(3.0)
    lo = np.floor(y).astype(int)
    fr = y - lo
    base = lo.min() - 3
    size = lo.max() - base + 5
    grid = np.zeros((size, 2))
    np.add.at(grid, lo - base, (1 - fr)[:, None] * v)
    np.add.at(grid, lo + 1 - base, fr[:, None] * v)
    mask = np.zeros(size)
    mask[lo - base] = 1
    mask[lo + 1 - base] = 1
    k = np.array([1, 2, 1]) / 4.0
    for _ in range(2):
        grid = np.stack([np.convolve(grid[:, c], k, mode="same") for c in range(2)], -1) * mask[:, None]
    want = (1 - fr)[:, None] * grid[lo - base] + fr[:, None] * grid[lo + 1 - base]
    np.testing.assert_allclose(out, want, atol=1e-6)
    assert nv == int(mask.sum())


def test_far_clusters_do_not_interact(oracle_lib):
    rng = np.random.default_rng(5)
    a = rng.normal(size=(50, 4)).astype(np.float32)
    b = (rng.normal(size=(50, 4)) + 100.0).astype(np.float32)
    va, vb = rng.normal(size=(50, 1)), rng.normal(size=(50, 1))
    both, _ = oracle_lib.lattice_filter(np.concatenate([a, b]), np.concatenate([va, vb]))
    np.testing.assert_allclose(both[:50], oracle_lib.lattice_filter(a, va)[0], rtol=1e-12)
    np.testing.assert_allclose(both[50:], oracle_lib.lattice_filter(b, vb)[0], rtol=1e-12)


def test_meanfield_update(oracle_lib):
    rng = np.random.default_rng(3)
    N, d, L = 200, 3, 4
    p = rng.normal(scale=1.5, size=(N, d)).astype(np.float32)
    U = rng.normal(size=(N, L))
    sm = lambda a: np.exp(a - a.max(1, keepdims=True)) / np.exp(a - a.max(1, keepdims=True)).sum(1, keepdims=True)
    np.testing.assert_allclose(oracle_lib.crf_meanfield(p, U, 0.0, 3), sm(-U), rtol=1e-12)
    Q1 = oracle_lib.crf_meanfield(p, U, 0.7, 1)
    F, _ = oracle_lib.lattice_filter(p, sm(-U))
    np.testing.assert_allclose(Q1, sm(-U + 0.7 * F), rtol=1e-12)
    Q3 = oracle_lib.crf_meanfield(p, U, 0.7, 3)
    np.testing.assert_allclose(Q3.sum(1), 1.0, atol=1e-12)


def test_meanfield_compatibility_matrix(oracle_lib):
    rng = np.random.default_rng(4)
    N, d, L = 150, 3, 5
    p = rng.normal(scale=1.5, size=(N, d)).astype(np.float32)
    U = rng.normal(size=(N, L))
    sm = lambda a: np.exp(a - a.max(1, keepdims=True)) / np.exp(a - a.max(1, keepdims=True)).sum(1, keepdims=True)
    np.testing.assert_allclose(oracle_lib.crf_meanfield_compat(p, U, np.zeros((L, L)), 2), sm(-U),
                               rtol=1e-12)
    w = 0.8
    potts = w * (1.0 - np.eye(L))
    for it in (1, 3):
        np.testing.assert_allclose(oracle_lib.crf_meanfield_compat(p, U, potts, it),
                                   oracle_lib.crf_meanfield(p, U, w, it), rtol=1e-10, atol=1e-13)
    # one isolated point, two labels, mu(0, 1) = a the only non-zero entry
    p1 = np.array([[0.3, -0.2, 0.1]], np.float32)
    u1 = np.array([[0.2, 0.9]])
    c = oracle_lib.lattice_filter(p1, np.ones((1, 1)))[0][0, 0]
    a = 1.7
    q = np.exp(-u1[0]) / np.exp(-u1[0]).sum()
    want = np.exp([-u1[0, 0] - a * c * q[1], -u1[0, 1]])
    want /= want.sum()
    got = oracle_lib.crf_meanfield_compat(p1, u1, np.array([[0.0, a], [0.0, 0.0]]), 1)
    np.testing.assert_allclose(got[0], want, rtol=1e-12)


@pytest.mark.parametrize("d", [1, 3, 6])
def test_filter_adjoint_identity(oracle_lib, d):
    rng = np.random.default_rng(40 + d)
    N, V = 300, 3
    p = rng.normal(scale=1.2, size=(N, d)).astype(np.float32)
    x = rng.normal(size=(N, V))
    y = rng.normal(size=(N, V))
    Fx, _ = oracle_lib.lattice_filter(p, x)
    Fty = oracle_lib.lattice_filter_adjoint(p, y)
    assert (Fx * y).sum() == pytest.approx((x * Fty).sum(), rel=1e-12)


def test_meanfield_compat_gradient_central_differences(oracle_lib):
    rng = np.random.default_rng(44)
    N, d, L, T = 60, 2, 3, 2
    p = rng.normal(scale=0.8, size=(N, d)).astype(np.float32)
    U = rng.normal(size=(N, L))
    mu = rng.normal(size=(L, L))
    gQ = rng.normal(size=(N, L))
    gu, gm = oracle_lib.crf_meanfield_compat_backward(p, U, mu, T, gQ)
    E = lambda U_, mu_: (gQ * oracle_lib.crf_meanfield_compat(p, U_, mu_, T)).sum()
    eps = 1e-6
    for l, k in [(0, 0), (0, 2), (2, 1), (1, 0)]:
        hi, lo = mu.copy(), mu.copy()
        hi[l, k] += eps
        lo[l, k] -= eps
        fd = (E(U, hi) - E(U, lo)) / (2 * eps)
        assert gm[l, k] == pytest.approx(fd, rel=1e-6, abs=1e-9), (l, k)
    for i, l in [(0, 0), (7, 2), (31, 1), (59, 0)]:
        hi, lo = U.copy(), U.copy()
        hi[i, l] += eps
        lo[i, l] -= eps
        fd = (E(hi, mu) - E(lo, mu)) / (2 * eps)
        assert gu[i, l] == pytest.approx(fd, rel=1e-6, abs=1e-9), (i, l)


def test_label_loss_kl_and_gradient(oracle_lib):
    """KL >= 0, zero iff softmax(logits) = Q; the gradient equals central
    differences of the loss and sums to zero over the labels (softmax is
    invariant to a common shift of the logits)."""
    rng = np.random.default_rng(9)
    N, L = 50, 6
    s = rng.normal(size=(N, L))
    Q = rng.dirichlet(np.ones(L), size=N)
    loss, g = oracle_lib.crf_label_loss(s, Q, 0.7)
    assert (loss >= 0).all()
    x = np.exp(s - s.max(1, keepdims=True))
    x /= x.sum(1, keepdims=True)
    np.testing.assert_allclose(loss, 0.7 * (x * np.log(x / Q)).sum(1), rtol=1e-12)
    z, _ = oracle_lib.crf_label_loss(np.log(Q) + 3.0, Q, 1.0)
    assert np.abs(z).max() < 1e-12
    np.testing.assert_allclose(g.sum(1), 0.0, atol=1e-12)
    for i, k in [(0, 0), (3, 5), (17, 2), (49, 4)]:
        hi, lo = s.copy(), s.copy()
        hi[i, k] += 1e-6
        lo[i, k] -= 1e-6
        fd = (oracle_lib.crf_label_loss(hi, Q, 0.7)[0][i] - oracle_lib.crf_label_loss(lo, Q, 0.7)[0][i]) / 2e-6
        assert fd == pytest.approx(g[i, k], rel=1e-6, abs=1e-9)


def test_property_loss(oracle_lib):
    """A constant property is its own filtered estimate (zero loss); for a
    random property the loss is |x - F(x)/F(1)|^2 with F the pinned filter,
    and the gradient 2 w (x - Q)."""
    rng = np.random.default_rng(4)
    p = rng.normal(scale=2.0, size=(300, 4)).astype(np.float32)
    const = np.tile([0.2, -0.5, 0.7], (300, 1))
    f, _ = oracle_lib.lattice_filter(p, np.concatenate([const, np.ones((300, 1))], 1))
    l0, g0 = oracle_lib.crf_property_loss(const, f, 2.0)
    assert np.abs(l0).max() < 1e-20 and np.abs(g0).max() < 1e-10
    x = rng.normal(size=(300, 3))
    f, _ = oracle_lib.lattice_filter(p, np.concatenate([x, np.ones((300, 1))], 1))
    loss, g = oracle_lib.crf_property_loss(x, f, 0.5)
    Q = f[:, :3] / f[:, 3:]
    np.testing.assert_allclose(loss, 0.5 * ((x - Q) ** 2).sum(1), rtol=1e-12)
    np.testing.assert_allclose(g, (x - Q), rtol=1e-12)


def test_surface_points_on_a_plane_and_sphere(oracle_lib):
    """A linear SDF (plane z = 0.3, f = 0.3 - z) is interpolated exactly, so
    the crossing lies on the plane; on the sphere grid the crossing of the
    central ray is within the interpolation error of radius 0.5; a ray that
    misses the grid reports no hit."""
    from synth import workloads
    from synth.scenes import voxel_positions
    from test_oracle_interp import _dense_blocks
    h = np.float32(1.0 / 16)
    blocks = _dense_blocks((-1, -1, -1), (0, 0, 0))
    pos = voxel_positions(blocks, float(h), np.zeros(3))
    vox = (-0.2 - pos[..., 2])[..., None]  # positive below the plane z = -0.2
    rays = np.array([[-0.2, 0.1, -0.8, 0.0, 0.0, 1.0], [0.1, -0.3, -0.9, 0.3, 0.2, 0.9327379],
                     [5.0, 5.0, 5.0, 1.0, 0.0, 0.0]], np.float32)
    params = {"step": float(h) / 2, "t_near": 0.0, "t_far": 3.0, "beta": float(h), "max_samples": 256}
    hit, pts, margin = oracle_lib.surface_points(blocks, vox, 0, h, np.zeros(3, np.float32), rays,
                                                 params)
    assert hit.tolist() == [True, True, False]
    np.testing.assert_allclose(pts[:2, 2], -0.2, atol=1e-6)
    assert (margin[:2] >= 0).all() and not pts[2].any()
    w = workloads.sphere_tiny()
    ray = w["rays"][(w["H"] // 2) * w["W"] + w["W"] // 2][None]
    hit, pts, _ = oracle_lib.surface_points(w["block_coords"], w["vox"], 3, w["h"], w["origin"], ray,
                                            w["params"])
    assert hit[0] and abs(np.linalg.norm(pts[0]) - 0.5) < 2e-3


def _lattice_vertex_volume(d):
    """Feature-space volume per vertex of the lattice, from its definition.

    The lattice is {x in Z^(d+1): sum x = 0, all x_i congruent mod d+1}; it
    has index (d+1)^(d-1) in A_d = {x in Z^(d+1): sum x = 0}, whose
    covolume is sqrt(d+1).  Features enter the plane sum x = 0 through an
    isometry times (d+1) sqrt(2/3), so a vertex owns
    sqrt(d+1) (d+1)^(d-1) / ((d+1) sqrt(2/3))^d = (3/2)^(d/2) / sqrt(d+1)
    of feature space."""
    return np.sqrt(d + 1.0) * (d + 1.0) ** (d - 1) / ((d + 1.0) * np.sqrt(2.0 / 3.0)) ** d


@pytest.mark.parametrize("d,N,A,margin", [(2, 50000, 8.0, 3.5), (3, 100000, 6.5, 3.5),
                                          (4, 300000, 5.0, 3.0), (6, 400000, 4.0, 2.5)])
def test_filter_is_an_isotropic_unit_gaussian(oracle_lib, d, N, A, margin):
    """Width and isotropy of the filter's Gaussian (Eq. 20, Sec. 3.5.3).

    Expected values, from the lattice alone: blurring with [1/4, 1/2, 1/4]
    along the d+1 steps u_j = (1,...,1) - (d+1) e_j adds the covariance
    (1/2) sum_j u_j u_j^T = ((d+1)^2 / 2) P (P the projector onto the
    plane).  Splatting onto the barycentric vertices of a simplex, and
    slicing from them, each add the vertex spread of the canonical simplex,
    (1/(d+2)) sum_k c_k c_k^T with c_k its vertices about their centroid,
    whose trace is (d+1)^2 d (d+2) / 12 and which averages over the
    simplices (permutations of one another) to ((d+1)^2 / 12) P.  Together
    (2/3)(d+1)^2 P: with features scaled by (d+1) sqrt(2/3) onto the plane
    that is the identity, a unit Gaussian in feature units.  A wrong factor
    on any axis makes the variance along that axis (or along random
    directions) differ from 1; a wrong common scale moves every variance and
    the mass.  The cloud is uniform, so the normalised moments at an interior
    point are the kernel's own; the bar (2 %) covers the sampling noise and
    the boundary and sparse-lattice effects (measured below 1 %)."""
    rng = np.random.default_rng(60 + d)
    p = rng.uniform(-A, A, size=(N, d)).astype(np.float32)
    P = p.astype(np.float64)
    dirs = [np.eye(d)[i] for i in range(d)]
    for _ in range(2):
        u = rng.normal(size=d)
        dirs.append(u / np.linalg.norm(u))
    vals = [np.ones(N)]
    for u in dirs:
        s = P @ u
        vals += [s, s * s]
    F, _ = oracle_lib.lattice_filter(p, np.stack(vals, 1))
    inner = (np.abs(P) < A - margin).all(1)
    assert inner.sum() > 1000
    mass = F[inner, 0].mean() / (N / (2 * A) ** d * _lattice_vertex_volume(d))
    assert abs(mass - 1.0) < 0.02, mass
    for j, u in enumerate(dirs):
        m1 = F[inner, 1 + 2 * j] / F[inner, 0]
        m2 = F[inner, 2 + 2 * j] / F[inner, 0]
        var = (m2 - m1 ** 2).mean()
        bias = (m1 - P[inner] @ u).mean()
        assert abs(var - 1.0) < 0.02, (j, var)
        assert abs(bias) < 0.02, (j, bias)
