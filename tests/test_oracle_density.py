"""Pins of the oracle's reduced density matrices (Alg. 1, step 5).

Each pin reaches the result by a route that shares nothing with the oracle's
pair-by-pair products: a closed form (the singlet), the free-fermion
correlation-matrix spectrum of the XX chain, the Schmidt decomposition, and the
dense partial trace through the brute-force index map.
"""
import itertools

import numpy as np
import pytest

import gen
from oracle import davidson, density, sectors

RANDOM_CASES = [(s, r) for s in range(6) for r in (1, 2)]


def _blocks_by_sector(prob):
    """(left sector, right sector, d_L, d_R) of every pair, in psi order."""
    table, _ = sectors.pair_table(prob.left, prob.right, prob.target)
    return [(sl, sr, dl, dr) for (sl, sr), (_, dl, dr) in table.items()]


def test_singlet_gives_maximally_mixed_spin():
    """Two spins in their singlet ground state: each spin's density matrix is
    1/2 times the identity (one state in each of the S^z = +-1/2 sectors)."""
    p = gen.heisenberg_exact(1, 1)
    E, psi, _ = davidson.ground_state_dense(p)
    assert E == pytest.approx(-0.75, abs=1e-14)
    left, right = density.density_sectors(p, psi)
    assert len(left) == 2
    for b in left + right:
        assert b.shape == (1, 1)
        assert b[0, 0] == pytest.approx(0.5, abs=1e-15)


def _xx_block_spectrum(nsites, nleft):
    """Peschel's free-fermion result for the open XX chain (Jordan-Wigner):
    the half-filled ground state's left-block density matrix has eigenvalues
    prod_j (n_j nu_j + (1 - n_j)(1 - nu_j)) over occupations n_j of the
    eigenmodes of the block's correlation matrix C_ij = <c_i^+ c_j> (nu_j its
    eigenvalues), with sum_j n_j = the block's particle number."""
    i = np.arange(1, nsites + 1)
    modes = [np.sqrt(2.0 / (nsites + 1)) * np.sin(k * np.pi * i / (nsites + 1)) for k in range(1, nsites + 1)]
    occ = modes[: nsites // 2]  # half filling; the other half differs by a sign pattern only
    C = sum(np.outer(f, f) for f in occ)[:nleft, :nleft]
    nu = np.linalg.eigvalsh(C)
    out = {}
    for n in itertools.product((0, 1), repeat=nleft):
        val = np.prod([nu[j] if n[j] else 1.0 - nu[j] for j in range(nleft)])
        out.setdefault(sum(n), []).append(val)
    return {k: np.sort(v) for k, v in out.items()}


@pytest.mark.parametrize("nl,nr", [(4, 4), (3, 5)])
def test_xx_chain_block_spectrum_matches_free_fermions(nl, nr):
    p = gen.heisenberg_exact(nl, nr, delta=0.0)
    _, psi, w = davidson.ground_state_dense(p)
    assert w[1] - w[0] > 1e-3  # non-degenerate ground state
    left, _ = density.density_sectors(p, psi)
    want = _xx_block_spectrum(nl + nr, nl)
    seen = set()
    for (sl, _, dl, _), blk in zip(_blocks_by_sector(p), left):
        lab = int(p.left.labels[sl, 0])  # 2 S^z = (#up - #down)
        nup = (lab + nl) // 2
        got = np.sort(np.linalg.eigvalsh(blk))
        ref = want[nup]
        # the spin-down-as-particle reading gives the same spectra (half filling)
        assert got.shape == ref.shape
        np.testing.assert_allclose(got, ref, atol=1e-12)
        seen.add(nup)
    assert seen == set(want.keys())


@pytest.mark.parametrize("seed,rank", RANDOM_CASES)
def test_schmidt_spectra_agree_and_trace_is_norm(seed, rank):
    """Schmidt decomposition: the non-zero eigenvalues of rho_L and rho_R are
    the same squared singular values, and both traces equal |psi|^2."""
    p = gen.random_problem(seed, rank=rank)
    psi = gen.start_vector(sectors.pair_table(p.left, p.right, p.target)[1], seed + 3)
    psi *= 1.7
    left, right = density.density_sectors(p, psi)
    nrm2 = float(psi @ psi)
    assert sum(np.trace(b) for b in left) == pytest.approx(nrm2, rel=1e-13)
    assert sum(np.trace(b) for b in right) == pytest.approx(nrm2, rel=1e-13)
    for bl, br, (_, _, dl, dr) in zip(left, right, _blocks_by_sector(p)):
        el, er = np.sort(np.linalg.eigvalsh(bl))[::-1], np.sort(np.linalg.eigvalsh(br))[::-1]
        r = min(dl, dr)
        np.testing.assert_allclose(el[:r], er[:r], atol=1e-12 * nrm2)
        assert np.all(np.abs(el[r:]) < 1e-12 * nrm2) and np.all(np.abs(er[r:]) < 1e-12 * nrm2)
        assert np.all(el[:r] > -1e-12 * nrm2)


@pytest.mark.parametrize("seed,rank", RANDOM_CASES)
def test_sector_blocks_match_dense_partial_trace(seed, rank):
    """The dense partial trace is block diagonal over sectors (charge
    conservation); its diagonal blocks are the pair blocks, zero for sectors
    that no pair of the target uses."""
    p = gen.random_problem(seed, rank=rank)
    psi = gen.start_vector(sectors.pair_table(p.left, p.right, p.target)[1], seed + 5)
    rL, rR = density.density_dense(p, psi)
    left, right = density.density_sectors(p, psi)
    offL, offR = p.left.offsets(), p.right.offsets()
    mask_l = np.zeros_like(rL, dtype=bool)
    mask_r = np.zeros_like(rR, dtype=bool)
    for (sl, sr, dl, dr), bl, br in zip(_blocks_by_sector(p), left, right):
        np.testing.assert_allclose(rL[offL[sl]:offL[sl + 1], offL[sl]:offL[sl + 1]], bl, atol=1e-14, rtol=1e-13)
        np.testing.assert_allclose(rR[offR[sr]:offR[sr + 1], offR[sr]:offR[sr + 1]], br, atol=1e-14, rtol=1e-13)
        mask_l[offL[sl]:offL[sl + 1], offL[sl]:offL[sl + 1]] = True
        mask_r[offR[sr]:offR[sr + 1], offR[sr]:offR[sr + 1]] = True
    assert np.all(rL[~mask_l] == 0.0) and np.all(rR[~mask_r] == 0.0)


def test_product_state_has_rank_one_density():
    """psi = u (x) v inside one pair: rank one, rho_L = |v|^2 u u^T and rho_R = |u|^2 v v^T."""
    p = gen.random_problem(2, rank=1)
    table, n = sectors.pair_table(p.left, p.right, p.target)
    (off, dl, dr) = max(table.values(), key=lambda t: t[1] * t[2])
    rng = np.random.default_rng(9)
    u, v = rng.standard_normal(dl), rng.standard_normal(dr)
    psi = np.zeros(n)
    psi[off:off + dl * dr] = np.outer(u, v).reshape(-1)
    left, right = density.density_sectors(p, psi)
    k = list(table.values()).index((off, dl, dr))
    np.testing.assert_allclose(left[k], (v @ v) * np.outer(u, u), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(right[k], (u @ u) * np.outer(v, v), rtol=1e-13, atol=1e-15)
    for j, b in enumerate(left):
        if j != k:
            assert np.all(b == 0.0)


def test_flat_layout_concatenates_pairs():
    p = gen.random_problem(4, rank=2)
    psi = gen.start_vector(sectors.pair_table(p.left, p.right, p.target)[1], 1)
    fl, fr = density.density_flat(p, psi)
    left, right = density.density_sectors(p, psi)
    assert fl.size == sum(b.size for b in left) and fr.size == sum(b.size for b in right)
    np.testing.assert_array_equal(fl[: left[0].size], left[0].reshape(-1))


# --------------------------------------------------------------------------- step 6


@pytest.mark.parametrize("seed,rank", RANDOM_CASES[:6])
def test_eigh_blocks_reconstructs_and_orders(seed, rank):
    """U diag(w) U^T = rho, U^T U = I, w descending, sign convention held."""
    p = gen.random_problem(seed, rank=rank, dmax=30)
    psi = gen.start_vector(sectors.pair_table(p.left, p.right, p.target)[1], seed)
    left, right = density.density_sectors(p, psi)
    vals, vecs = density.eigh_blocks(left + right)
    for B, w, U in zip(left + right, vals, vecs):
        d = B.shape[0]
        scale = max(np.abs(B).max(), 1e-300)
        np.testing.assert_allclose(U @ np.diag(w) @ U.T, B, atol=1e-13 * scale * d)
        np.testing.assert_allclose(U.T @ U, np.eye(d), atol=1e-13 * d)
        assert np.all(np.diff(w) <= 0)
        for j in range(d):
            k = int(np.argmax(np.abs(U[:, j])))
            assert U[k, j] > 0


def test_eigh_blocks_xx_chain_spectrum():
    """The free-fermion spectra of the XX chain's left block, through the
    oracle's step-6 routine."""
    p = gen.heisenberg_exact(4, 4, delta=0.0)
    _, psi, _ = davidson.ground_state_dense(p)
    left, _ = density.density_sectors(p, psi)
    vals, _ = density.eigh_blocks(left)
    want = _xx_block_spectrum(8, 4)
    for (sl, _, _, _), w in zip(_blocks_by_sector(p), vals):
        nup = (int(p.left.labels[sl, 0]) + 4) // 2
        np.testing.assert_allclose(w, want[nup][::-1], atol=1e-12)


# --------------------------------------------------------------------------- step 7 (selection)


def test_truncation_weight_is_the_projection_error():
    """Keeping the left block's states of largest weight: the discarded weight
    equals |psi - P psi|^2 with P the projector on the kept eigenvectors, and it
    is the smallest such error over the same number of states (here checked
    against keeping the states of smallest weight instead)."""
    p = gen.random_problem(7, rank=1, dmax=14)
    psi = gen.start_vector(sectors.pair_table(p.left, p.right, p.target)[1], 4)
    psi /= np.linalg.norm(psi)
    table, _ = sectors.pair_table(p.left, p.right, p.target)
    left, _ = density.density_sectors(p, psi)
    vals, vecs = density.eigh_blocks(left)
    total = sum(len(v) for v in vals)
    for m in (1, 3, total // 2, total - 1, total, total + 5):
        counts, disc = density.truncate(vals, m)
        assert counts.sum() == min(m, total)
        err = alt = 0.0
        for (off, dl, dr), U, k in zip(table.values(), vecs, counts):
            X = psi[off:off + dl * dr].reshape(dl, dr)
            P = U[:, :k] @ U[:, :k].T
            err += float(np.sum((X - P @ X) ** 2))
            Q = U[:, dl - k:] @ U[:, dl - k:].T  # the same counts, states of smallest weight
            alt += float(np.sum((X - Q @ X) ** 2))
        assert disc == pytest.approx(err, abs=1e-13)
        assert alt >= err - 1e-13


def test_truncation_of_xx_chain_matches_free_fermion_weights():
    p = gen.heisenberg_exact(4, 4, delta=0.0)
    _, psi, _ = davidson.ground_state_dense(p)
    vals, _ = density.eigh_blocks(density.density_sectors(p, psi)[0])
    spec = np.sort(np.concatenate(list(_xx_block_spectrum(8, 4).values())))[::-1]
    for m in (2, 5, 9):
        counts, disc = density.truncate(vals, m)
        assert counts.sum() == m
        assert disc == pytest.approx(float(spec[m:].sum()), abs=1e-12)


def test_truncation_ties_follow_block_order():
    vals = [np.array([0.4, 0.1]), np.array([0.4, 0.1]), np.array([0.0])]
    assert density.truncate(vals, 1)[0].tolist() == [1, 0, 0]
    assert density.truncate(vals, 3)[0].tolist() == [2, 1, 0]
    c, d = density.truncate(vals, 0)
    assert c.tolist() == [0, 0, 0] and d == pytest.approx(1.0)


# --------------------------------------------------------------------------- step 7 (operators)


def test_renormalized_identity_and_own_eigenbasis():
    """The identity stays the identity on the kept states (U has orthonormal
    columns); a symmetric block taken to its own eigenbasis is diagonal with
    its eigenvalues."""
    rng = np.random.default_rng(2)
    G = rng.standard_normal((9, 9))
    H = (G + G.T) / 2
    vals, vecs = density.eigh_blocks([H])
    U = vecs[0]
    np.testing.assert_allclose(density.renormalize_block(np.ones(9), U, U, 4, 4), np.eye(4), atol=1e-14)
    np.testing.assert_allclose(density.renormalize_block(H, U, U, 9, 6), np.diag(vals[0])[:, :6], atol=1e-13)


def test_renormalized_superblock_is_the_projected_superblock():
    """The basis change of one block: with V = blockdiag over sectors of the
    kept eigenvectors of rho_L, every left operator renormalized block by block
    gives the superblock Hamiltonian V^T H V (V acting on the left block only,
    dense Kronecker products), and the truncated state V^T psi keeps the
    weight 1 - discarded."""
    p = gen.heisenberg_exact(3, 3)
    _, psi, _ = davidson.ground_state_dense(p)
    left, _ = density.density_sectors(p, psi)
    vals, vecs = density.eigh_blocks(left)
    counts, disc = density.truncate(vals, 4)
    table, _ = sectors.pair_table(p.left, p.right, p.target)
    kept = {sl: (vecs[i], int(counts[i])) for i, ((sl, _), _) in enumerate(table.items())}
    off = p.left.offsets()
    mL = p.left.m
    # V: full left space -> kept states, sector by sector in sector order
    cols = []
    for s in range(p.left.nsec):
        if s in kept:
            U, k = kept[s]
            for j in range(k):
                c = np.zeros(mL)
                c[off[s]:off[s + 1]] = U[:, j]
                cols.append(c)
    V = np.array(cols).T
    for op in p.ops_left:
        A = sectors.dense_operator(p.left, op)
        want = V.T @ A @ V
        got = np.zeros_like(want)
        new_off = {}
        pos = 0
        for s in range(p.left.nsec):
            if s in kept:
                new_off[s] = pos
                pos += kept[s][1]
        for s in kept:
            for t in kept:
                blk = A[off[t]:off[t + 1], off[s]:off[s + 1]]
                got[new_off[t]:new_off[t] + kept[t][1], new_off[s]:new_off[s] + kept[s][1]] = \
                    density.renormalize_block(blk, kept[t][0], kept[s][0], kept[t][1], kept[s][1])
        np.testing.assert_allclose(got, want, atol=1e-13)
    full = np.zeros(mL * p.right.m)
    full[sectors.layout(p.left, p.right, p.target).index_map] = psi
    red = V.T @ full.reshape(mL, p.right.m)
    assert float(np.sum(red ** 2)) == pytest.approx(1.0 - disc, abs=1e-13)
