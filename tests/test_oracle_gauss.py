"""Pins of the oracle's Gaussian medium and local KL parametrization (Sec.
5.3 with Sec. 2.1's local KL, eqs. localKL and local_KL_truncation): the
paper's fallback probability, the spectral field's variance and covariance
against eq. betaCov (Monte Carlo), the dense local KL against the separable
product of one-dimensional eigenproblems, orthonormal modes and the trace,
exact recovery of synthesized parameters, the mean truncation error against
the discarded eigenvalues, and the fallback rate of the spectral field."""
import numpy as np
import pytest

from oracle import gauss
from paper_1607_00693_amd import workloads as W


def test_fallback_probability_is_the_papers():
    # Sec. 5.3: four local parameters, box [-3, 3], interpolation used with
    # probability 0.9892 and the fine solve with probability 0.0108
    assert round(gauss.outside_probability(4, 3.0), 4) == 0.0108
    assert round(1 - gauss.outside_probability(4, 3.0), 4) == 0.9892


def test_spectral_field_has_the_gaussian_covariance():
    l1, l2, nf, N = 0.5, 0.1, 32, 600
    z, u = W.spectral_draws(N, 128, 71)
    b = gauss.field(z, u, nf, l1, l2)
    se = np.sqrt(2.0 / N)
    assert abs(b.var(axis=0).mean() - 1.0) < 4.5 * se / 8  # averaged over the grid
    assert abs(b.mean()) < 0.1
    h = 1.0 / nf
    for d in (1, 2, 4):
        cx = (b[:, :, :-d] * b[:, :, d:]).mean()
        cy = (b[:, :-d, :] * b[:, d:, :]).mean()
        assert abs(cx - np.exp(-(d * h) ** 2 / l1**2)) < 0.1
        assert abs(cy - np.exp(-(d * h) ** 2 / l2**2)) < 0.1


def test_spectral_field_covariance_is_exact_under_quadrature():
    # the covariance of one cosine term, averaged over its phase and over
    # its wave vector, is E_w[cos(w . d)] = exp(-|d|^2 / l^2) exactly when w
    # has the normal law N(0, 2/l^2) per component.  Replacing the random
    # draws by a Gauss-Hermite rule in z (40 nodes, exact to rounding for
    # this smooth integrand) and four equispaced phases (the phase average of
    # cos(a + p) cos(b + p) is cos(a - b) / 2 exactly) makes the check
    # deterministic, so any slip in the scaling of the wave vectors (a
    # factor sqrt 2, l1 and l2 swapped) shows at every lag
    l1, l2, nf = 0.5, 0.1, 32
    zn, zw = np.polynomial.hermite_e.hermegauss(40)
    zw = zw / np.sqrt(2.0 * np.pi)
    phases = np.arange(4) / 4.0
    h = 1.0 / nf
    for axis, l in ((0, l1), (1, l2)):
        z = np.zeros((len(zn) * 4, 1, 2))
        u = np.zeros((len(zn) * 4, 1))
        wts = np.zeros(len(zn) * 4)
        for k in range(len(zn)):
            for p in range(4):
                z[4 * k + p, 0, axis] = zn[k]
                u[4 * k + p, 0] = phases[p]
                wts[4 * k + p] = zw[k] / 4.0
        b = gauss.field(z, u, nf, l1, l2)  # one term: J = 1
        line = b[:, 5, :] if axis == 0 else b[:, :, 7]
        assert abs(np.einsum("s,sx->x", wts, line * line).max() - 1.0) < 1e-12
        for d in range(1, 12):
            cov = np.einsum("s,sx->x", wts, line[:, :-d] * line[:, d:])
            assert np.abs(cov - np.exp(-(d * h) ** 2 / l**2)).max() < 1e-12, (axis, d)


def test_local_kl_is_the_separable_product():
    m, h, l1, l2 = 12, 1.0 / 96, 1.0, 1.0 / 48
    mu, V, frac = gauss.local_kl(m, h, l1, l2, 8)
    c = (np.arange(m) + 0.5) * h
    ex = np.linalg.eigvalsh(np.exp(-((c[:, None] - c[None, :]) ** 2) / l1**2))
    ey = np.linalg.eigvalsh(np.exp(-((c[:, None] - c[None, :]) ** 2) / l2**2))
    prod = np.sort(np.outer(ex, ey).ravel())[::-1]
    np.testing.assert_allclose(mu, prod[:8], rtol=1e-10, atol=1e-12 * prod[0])
    G = V.reshape(8, -1) @ V.reshape(8, -1).T
    np.testing.assert_allclose(G, np.eye(8), atol=1e-12)
    assert abs(prod.sum() - m * m) < 1e-9 * m * m  # unit variance: trace = m^2
    assert 0.99 < frac < 1.0


def test_projection_recovers_synthesized_parameters():
    nc, m, K = 3, 8, 5
    mu, V, _ = gauss.local_kl(m, 1.0 / (nc * m), 1.0, 1.0 / 48, K)
    xi = np.random.default_rng(3).normal(size=(2, nc * nc, K))
    beta = np.zeros((2, nc * m, nc * m))
    for ky in range(nc):
        for kx in range(nc):
            beta[:, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m] = np.einsum(
                "nk,kij->nij", xi[:, ky * nc + kx] * np.sqrt(mu), V)
    np.testing.assert_allclose(gauss.project(beta, nc, m, mu, V), xi, rtol=0, atol=1e-12)


def test_projection_on_oversampled_patches():
    # patches of side m + 2o around each element, moved inside the domain:
    # with nc = 4, m = 8, o = 4 the patch origins along an axis are 0, 4, 12,
    # 16 (elements 0 and 3 are pushed in from -4 and 20).  Parameters
    # synthesized on one element's patch (random field elsewhere) come back,
    # which a wrong origin or a transposed patch would break; o = 0 is the
    # element projection.
    nc, m, o, K = 4, 8, 4, 5
    P, nf = m + 2 * o, nc * m
    mu, V, _ = gauss.local_kl(P, 1.0 / nf, 1.0, 1.0 / 24, K)
    rng = np.random.default_rng(5)
    for (kx, ky), (x0, y0) in {(0, 0): (0, 0), (1, 2): (4, 12), (3, 1): (16, 4), (2, 3): (12, 16)}.items():
        beta = rng.normal(size=(2, nf, nf))
        xs = rng.normal(size=(2, K))
        beta[:, y0:y0 + P, x0:x0 + P] = np.einsum("nk,kij->nij", xs * np.sqrt(mu), V)
        xi = gauss.project_patches(beta, nc, m, o, mu, V)
        np.testing.assert_allclose(xi[:, ky * nc + kx], xs, rtol=0, atol=1e-12)
    mu0, V0, _ = gauss.local_kl(m, 1.0 / nf, 1.0, 1.0 / 24, K)
    beta = rng.normal(size=(2, nf, nf))
    np.testing.assert_allclose(gauss.project_patches(beta, nc, m, 0, mu0, V0), gauss.project(beta, nc, m, mu0, V0),
                               rtol=0, atol=1e-13)
    with pytest.raises(ValueError):
        gauss.project_patches(beta, 1, m, o, mu, V)


def test_oversampled_patch_kl_in_the_papers_geometry():
    # Sec. 5.3: the local KL on the oversampled domain of side 2H with l2 = H
    # (two correlation lengths across), four terms.  The kept fraction of the
    # patch variance and the rate of pairs with a parameter outside [-3, 3]
    # against 1 - P(|Z| <= 3)^4 = 0.0108 on spectral samples.
    nc, m = 8, 8
    o = m // 2
    P, nf = m + 2 * o, nc * m
    l1, l2 = 1.0, 1.0 / nc
    mu, V, cap = gauss.local_kl(P, 1.0 / nf, l1, l2, 4)
    assert 0.985 < mu.sum() / (P * P) < 0.997  # four terms keep roughly 99% (Sec. 5.3)
    N = 100
    z, u = W.spectral_draws(N, 256, 73)
    xi = gauss.project_patches(gauss.field(z, u, nf, l1, l2), nc, m, o, mu, V)
    out = (np.abs(xi) > 3.0).any(axis=2)
    p = gauss.outside_probability(4)
    assert abs(out.mean() - p) < 4.5 * np.sqrt(p * (1 - p) / out.size) + 0.003


def test_truncation_error_matches_the_discarded_spectrum_and_the_fallback_rate():
    wl = W.GAUSS16
    nc, m = 8, wl.m  # half the mesh, same element size and correlation lengths
    nf = nc * m
    # the workload's correlation lengths in element units, on a mesh of nc x nc elements of [0, 1]
    l1, l2 = wl.l1 * wl.nc / nc, wl.l2 * wl.nc / nc
    mu_all, V_all, _ = gauss.local_kl(m, 1.0 / nf, l1, l2, 8)
    N = 120
    z, u = W.spectral_draws(N, wl.nterms, 72)
    beta = gauss.field(z, u, nf, l1, l2)
    xi_all = gauss.project(beta, nc, m, mu_all, V_all)
    # mean squared truncation error of beta per patch = sum of the discarded mu
    for K in (2, 4, 6):
        b_K = np.einsum("npk,kij->npij", xi_all[:, :, :K] * np.sqrt(mu_all[:K]), V_all[:K])
        blocks = np.stack([beta[:, ky * m:(ky + 1) * m, kx * m:(kx + 1) * m]
                           for ky in range(nc) for kx in range(nc)], axis=1)
        mse = ((blocks - b_K) ** 2).sum(axis=(2, 3)).mean()
        ref = m * m - mu_all[:K].sum()  # trace (unit variance) minus the kept part
        assert abs(mse - ref) < 0.15 * ref + 1e-12, (K, mse, ref)
    # pairs with a parameter outside [-3, 3] among the first four
    out = (np.abs(xi_all[:, :, :4]) > 3.0).any(axis=2)
    p = gauss.outside_probability(4)
    n = out.size
    assert abs(out.mean() - p) < 4.5 * np.sqrt(p * (1 - p) / n) + 0.003


def test_interpolation_on_the_local_parameters():
    # the table interpolant converges to the truncated-coefficient S inside
    # the box, the interpolation error stays below the truncation error (the
    # paper's observation in Sec. 5.3), and out-of-box pairs are the plain
    # solve of the sample's own coefficient
    from oracle import core
    nc, m, K = 4, 8, 4
    nf = nc * m
    l1, l2 = 1.0, 2.0 / (nc * 2 * 2)  # two correlation lengths per element, as in the workload
    mu, V, _ = gauss.local_kl(m, 1.0 / nf, l1, l2, K)
    z, u = W.spectral_draws(6, 128, 73)
    beta = gauss.field(z, u, nf, l1, l2)
    kap = gauss.kappa(beta)
    xi = gauss.project(beta, nc, m, mu, V)
    S_trunc, _, _ = core.upscale(gauss.truncated_kappa_blocks(xi, mu, V, K).reshape(-1, m, m), 1, 1, m)
    S_trunc = S_trunc.reshape(6, nc * nc, 10)
    S_full, _, _ = core.upscale(kap, nc, nc, m)
    err = {}
    for nn in (3, 5, 7):
        model = gauss.kl_interp_offline(m, mu, V, nn)
        S, fb = gauss.kl_interp_online(model, xi, kap, nc, m)
        ins = ~fb
        sc = np.abs(S_full).max(axis=2)
        err[nn] = (np.abs(S - S_trunc).max(axis=2)[ins] / sc[ins]).max()
        if fb.any():
            np.testing.assert_array_equal(S[fb], S_full[fb])
    assert err[3] > err[5] > err[7], err
    trunc = (np.abs(S_trunc - S_full).max(axis=2) / np.abs(S_full).max(axis=2))[~fb].max()
    assert err[7] < 0.1 * trunc, (err[7], trunc)


def test_oversampled_stiffness_depends_on_the_patch_and_its_class_only():
    # the oversampled stiffness of an element, computed on the whole field,
    # equals the one of its patch placed in a 3 x 3-element mesh at the
    # element's class (corner, edge, interior elements): the embedding the
    # interpolation tables are built on
    from oracle import core
    nc, m, o = 4, 8, 4
    P, nf = m + 2 * o, nc * m
    a = np.exp(np.random.default_rng(11).normal(size=(nf, nf)))
    assert [gauss.element_class(k, m, o, nc) for k in range(nc)] == [0, 1, 1, 2]
    for kx, ky in [(0, 0), (1, 2), (3, 3), (2, 0), (3, 1)]:
        x0, y0 = gauss.patch_origin(kx, m, o, nf), gauss.patch_origin(ky, m, o, nf)
        full = core.cell_S_os(a, m, o, kx, ky).ravel()
        emb = gauss.os_S_embedded(a[None, y0:y0 + P, x0:x0 + P], m, o, gauss.element_class(kx, m, o, nc),
                                  gauss.element_class(ky, m, o, nc))[0]
        np.testing.assert_allclose(emb, full, rtol=0, atol=1e-12 * np.abs(full).max())


def test_oversampled_interpolation_in_the_patch_parameters():
    # nodal exactness (the interpolant at a node is the oversampled stiffness
    # of the truncated coefficient there, on the real mesh), convergence in
    # the number of nodes, and the sample's own stiffness outside the box
    from oracle import core
    nc, m, o, K = 4, 8, 4, 3
    P, nf = m + 2 * o, nc * m
    mu, V, _ = gauss.local_kl(P, 1.0 / nf, 1.0, 1.0 / 8, K)
    models = {nn: gauss.kl_interp_os_offline(m, o, mu, V, nn, box=2.0) for nn in (3, 5)}
    nodes = models[3]["nodes"]
    # a node's parameters on element (1, 2): its patch carries the truncated KL
    xn = np.array([nodes[0], nodes[1], nodes[2]])
    blk = gauss.truncated_kappa_blocks(xn[None, None], mu, V, K)[0, 0]
    a = np.ones((nf, nf))
    x0, y0 = gauss.patch_origin(1, m, o, nf), gauss.patch_origin(2, m, o, nf)
    a[y0:y0 + P, x0:x0 + P] = blk
    xi = np.zeros((1, nc * nc, K))
    xi[0, 2 * nc + 1] = xn
    S, fb = gauss.kl_interp_os_online(models[3], xi, a[None], nc)
    ref = core.cell_S_os(a, m, o, 1, 2).ravel()
    np.testing.assert_allclose(S[0, 2 * nc + 1], ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    # convergence at random parameters inside the box, interior and corner classes
    rng = np.random.default_rng(12)
    xr = rng.uniform(-2.0, 2.0, size=(6, K))
    blocks = gauss.truncated_kappa_blocks(xr[:, None], mu, V, K)[:, 0]
    err = {}
    for nn, md in models.items():
        e = 0.0
        for cls in [(1, 1), (0, 2)]:
            ref = gauss.os_S_embedded(blocks, m, o, *cls)
            from oracle import ri
            got = ri.ri_eval(md["tables"][cls], md["nodes"], xr)
            e = max(e, float((np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max()))
        err[nn] = e
    assert err[5] < 0.2 * err[3] and err[5] < 1e-2, err
    # outside the box: the sample's own oversampled stiffness
    xi_out = np.full((1, nc * nc, K), 5.0)
    a2 = np.exp(rng.normal(size=(1, nf, nf)))
    S2, fb2 = gauss.kl_interp_os_online(models[3], xi_out, a2, nc)
    assert fb2.all()
    S_ref, _ = core.upscale_os(a2, nc, nc, m, o)
    np.testing.assert_allclose(S2, S_ref, rtol=0, atol=1e-12 * np.abs(S_ref).max())


def test_oversampled_sparse_grid_interpolation():
    # the Smolyak interpolant on the sparse grid of the patch parameters:
    # nodal exactness against the oversampled stiffness of the truncated
    # coefficient, and convergence from level 2 to level 4 (29 -> 137 ->
    # ... nodes in 3 variables) at random points, for an interior and a
    # corner class
    from oracle import ri, sc
    nc, m, o, K = 4, 8, 4, 3
    P, nf = m + 2 * o, nc * m
    mu, V, _ = gauss.local_kl(P, 1.0 / nf, 1.0, 1.0 / 8, K)
    box = 2.0
    md = {L: gauss.kl_sgi_os_offline(m, o, mu, V, L, box) for L in (2, 3, 4)}
    dg, _ = sc.sparse_grid(K, 3)
    r = 7
    x = np.array([sc.node_values(dg[r:r + 1, i], 3, -box, box)[0] for i in range(K)])
    blk = gauss.truncated_kappa_blocks(x[None, None], mu, V, K)[:, 0]
    for cls in [(1, 1), (0, 2)]:
        ref = gauss.os_S_embedded(blk, m, o, *cls)[0]
        got = sc.smolyak_interp(md[3]["tables"][cls], K, 3, (x / box)[None])[0]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    xr = np.random.default_rng(13).uniform(-box, box, size=(6, K))
    blocks = gauss.truncated_kappa_blocks(xr[:, None], mu, V, K)[:, 0]
    err = {}
    for L, model in md.items():
        e = 0.0
        for cls in [(1, 1), (0, 2)]:
            ref = gauss.os_S_embedded(blocks, m, o, *cls)
            got = sc.smolyak_interp(model["tables"][cls], K, L, xr / box)
            e = max(e, float((np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max()))
        err[L] = e
    assert err[4] < 0.3 * err[2] and err[4] < 1e-2, err
    # online: interior pairs through the sparse tables, the rest as before
    xi = np.zeros((1, nc * nc, K))
    xi[0, 5] = x
    xi[0, 6] = 3.0
    a = np.exp(np.random.default_rng(14).normal(size=(1, nf, nf)))
    S, fb = gauss.kl_interp_os_online(md[3], xi, a, nc)
    assert fb[0, 6] and not fb[0, 5]
    ref = gauss.os_S_embedded(blk, m, o, gauss.element_class(1, m, o, nc), gauss.element_class(1, m, o, nc))[0]
    np.testing.assert_allclose(S[0, 5], ref, rtol=0, atol=1e-11 * np.abs(ref).max())
