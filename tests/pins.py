"""Pins for the CPU oracle: checks against facts the mathematics fixes, none of
which re-types the oracle's own formulas.

Each ``pin_*`` takes an oracle module ``O`` (the real one, or one with a
planted mistake) and raises ``AssertionError`` when the oracle disagrees with
the fact.  The real oracle must pass all of them; every planted mistake must
fail at least one (see ``test_oracle_mutants.py``).

Facts used (derivations are in the docstrings):
* brute force: pure-Python loops over the 4-index integrals, written from the
  paper's printed index forms (Eq. MP2_ints and the Appendix definitions of
  X, Gamma, D_ij and D_ab), on tiny inputs;
* a closed form for nocc = nvir = 1;
* equal orbital energies, where E reduces to Gram-matrix traces;
* dE/dB = 4 Gamma (the factor of the Appendix's Z = 4 Gamma + ...), checked by
  complex-step differentiation;
* dE/d eps_i = 2 (P_ij)_ii and dE/d eps_a = 2 (P_ab)_aa, complex step;
* symmetry, trace and sign properties, orthogonal rotation of the auxiliary
  index, global shift of all orbital energies, scaling of B, zero padding and
  index permutation;
* pair screening: screening out every pair that contains occupied orbital i
  gives the results of the fragment with orbital i deleted (zero in row and
  column i), and a mask names unordered pairs.
"""
from __future__ import annotations

import numpy as np

RTOL = 1e-12


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den)


def tiny_inputs(nocc, nvir, naux, seed, complex_ok=False):
    rng = np.random.default_rng(seed)
    B = 0.3 * rng.standard_normal((nocc, nvir, naux)) * np.exp(-np.arange(naux) / 7.0)
    eo = np.sort(rng.uniform(-20.0, -0.3, nocc))
    ev = np.sort(rng.uniform(0.1, 5.0, nvir))
    return B, eo, ev


def brute_force(B, eo, ev):
    """All outputs from pure-Python loops over the paper's index forms."""
    nocc, nvir, naux = B.shape
    I = {}
    for i in range(nocc):
        for a in range(nvir):
            for j in range(nocc):
                for b in range(nvir):
                    s = 0.0
                    for P in range(naux):
                        s += B[i, a, P] * B[j, b, P]
                    I[i, a, j, b] = s

    def D(i, j, a, b):
        return eo[i] + eo[j] - ev[a] - ev[b]

    X = {(i, j, a, b): I[i, a, j, b] / D(i, j, a, b)
         for i in range(nocc) for j in range(nocc) for a in range(nvir) for b in range(nvir)}
    E = 0.0
    e_pair = np.zeros((nocc, nocc))
    for i in range(nocc):
        for j in range(nocc):
            s = 0.0
            for a in range(nvir):
                for b in range(nvir):
                    s += I[i, a, j, b] * (2 * I[i, a, j, b] - I[i, b, j, a]) / D(i, j, a, b)
            e_pair[i, j] = s
            E += s
    G = np.zeros((nocc, nvir, naux))
    for i in range(nocc):
        for a in range(nvir):
            for P in range(naux):
                s = 0.0
                for j in range(nocc):
                    for b in range(nvir):
                        s += (2 * X[i, j, a, b] - X[i, j, b, a]) * B[j, b, P]
                G[i, a, P] = s
    Pij = np.zeros((nocc, nocc))
    for i in range(nocc):
        for j in range(nocc):
            s = 0.0
            for a in range(nvir):
                for b in range(nvir):
                    for k in range(nocc):
                        s += (2 * X[i, k, a, b] - X[k, i, a, b]) * X[j, k, a, b]
            Pij[i, j] = -s
    Pab = np.zeros((nvir, nvir))
    for a in range(nvir):
        for b in range(nvir):
            s = 0.0
            for i in range(nocc):
                for j in range(nocc):
                    for c in range(nvir):
                        s += (2 * X[i, j, a, c] - X[i, j, c, a]) * X[i, j, b, c]
            Pab[a, b] = s
    return dict(E=E, e_pair=e_pair, Gamma=G, P_ij=Pij, P_ab=Pab)


def pin_brute_force(O, shapes=((2, 3, 4), (3, 4, 5), (1, 5, 3), (4, 2, 6))):
    for n, (nocc, nvir, naux) in enumerate(shapes):
        B, eo, ev = tiny_inputs(nocc, nvir, naux, 10 + n)
        r = O.fragment(B, eo, ev)
        bf = brute_force(B, eo, ev)
        assert abs(r["E"] - bf["E"]) <= 1e-13 * abs(bf["E"]), ("E", r["E"], bf["E"])
        for key in ("e_pair", "Gamma", "P_ij", "P_ab"):
            assert rel(r[key], bf[key]) <= 1e-13, (key, rel(r[key], bf[key]))


def pin_closed_form_single_pair(O):
    """nocc = nvir = 1: V = sum_P B_P^2, D = 2(eps_i - eps_a), X = V / D,
    T = 2X - X = X, so E = V^2 / D, Gamma_P = X B_P, P_ij = -X^2, P_ab = X^2."""
    rng = np.random.default_rng(3)
    for naux in (1, 2, 7):
        Bv = rng.standard_normal(naux)
        ei, ea = -1.3, 0.7
        r = O.fragment(Bv.reshape(1, 1, naux), np.array([ei]), np.array([ea]))
        V = float(np.dot(Bv, Bv))
        D = 2.0 * (ei - ea)
        X = V / D
        assert abs(r["E"] - V * V / D) <= 1e-14 * abs(V * V / D)
        assert rel(r["Gamma"].ravel(), X * Bv) <= 1e-14
        assert abs(r["P_ij"][0, 0] + X * X) <= 1e-14 * X * X
        assert abs(r["P_ab"][0, 0] - X * X) <= 1e-14 * X * X


def pin_equal_energies(O):
    """All eps_i = e_o and all eps_a = e_v: every D equals 2(e_o - e_v), so
    E = [2 sum (ia|jb)^2 - sum (ia|jb)(ib|ja)] / (2(e_o - e_v)).  With the
    matrix M[(i,a), P] = B^P_ia and G = M^T M (naux x naux Gram matrix),
    sum (ia|jb)^2 = tr(G^2); with W_ij = B_i^T B_j (naux x naux, a contraction
    over the orbital index first instead of the auxiliary index) and
    W_ji = W_ij^T, the exchange sum is sum_ij sum_PQ W_ij[P,Q] W_ji[P,Q] =
    sum_ij tr(W_ij W_ij)."""
    for nocc, nvir, naux in ((3, 4, 5), (2, 7, 3)):
        B, _, _ = tiny_inputs(nocc, nvir, naux, 21 + nocc)
        eo_v, ev_v = -2.5, 1.25
        eo = np.full(nocc, eo_v)
        ev = np.full(nvir, ev_v)
        M = B.reshape(nocc * nvir, naux)
        G = M.T @ M
        coul = np.trace(G @ G)
        exch = 0.0
        for i in range(nocc):
            for j in range(nocc):
                W = B[i].T @ B[j]
                exch += np.trace(W @ W)
        E_ref = (2.0 * coul - exch) / (2.0 * (eo_v - ev_v))
        r = O.fragment(B, eo, ev)
        assert abs(r["E"] - E_ref) <= 1e-13 * abs(E_ref), (r["E"], E_ref)


def _complex_E(O, B, eo, ev):
    return O.fragment(B, eo, ev, gamma=False, density=False)["E"]


def pin_dE_dB_is_4_gamma(O):
    """dE/dB^P_ia = 4 Gamma^P_ia, every element, by complex step (h = 1e-30):
    Im E(B + i h e_n) / h equals the derivative to rounding."""
    h = 1e-30
    for nocc, nvir, naux in ((2, 3, 3), (3, 2, 4)):
        B, eo, ev = tiny_inputs(nocc, nvir, naux, 31 + naux)
        G = O.fragment(B, eo, ev)["Gamma"]
        dE = np.zeros_like(B)
        for idx in np.ndindex(B.shape):
            Bc = B.astype(np.complex128)
            Bc[idx] += 1j * h
            dE[idx] = _complex_E(O, Bc, eo, ev).imag / h
        assert rel(dE, 4.0 * G) <= 1e-12, rel(dE, 4.0 * G)


def pin_dE_deps_is_2_diagP(O):
    """dE/d eps_i = 2 (P_ij)_ii and dE/d eps_a = 2 (P_ab)_aa (complex step)."""
    h = 1e-30
    B, eo, ev = tiny_inputs(3, 4, 5, 41)
    r = O.fragment(B, eo, ev)
    for i in range(len(eo)):
        e = eo.astype(np.complex128)
        e[i] += 1j * h
        d = _complex_E(O, B, e, ev).imag / h
        assert abs(d - 2.0 * r["P_ij"][i, i]) <= 1e-12 * abs(d), (i, d, r["P_ij"][i, i])
    for a in range(len(ev)):
        e = ev.astype(np.complex128)
        e[a] += 1j * h
        d = _complex_E(O, B, eo, e).imag / h
        assert abs(d - 2.0 * r["P_ab"][a, a]) <= 1e-12 * abs(d), (a, d, r["P_ab"][a, a])


def pin_symmetry_and_sign(O):
    """e_ij = e_ji <= 0 (with W = 1/|D| symmetric in a, b,
    sum W V V^T <= sum W V^2 by Cauchy-Schwarz), E <= 0, P_ij and P_ab
    symmetric, tr P_ij + tr P_ab = 0, tr P_ab >= 0."""
    B, eo, ev = tiny_inputs(5, 6, 8, 51)
    r = O.fragment(B, eo, ev)
    ep = r["e_pair"]
    assert rel(ep, ep.T) <= 1e-13
    assert np.all(ep <= 0.0) and r["E"] <= 0.0
    assert rel(r["P_ij"], r["P_ij"].T) <= 1e-13
    assert rel(r["P_ab"], r["P_ab"].T) <= 1e-13
    tij, tab = np.trace(r["P_ij"]), np.trace(r["P_ab"])
    assert tab >= 0.0
    assert abs(tij + tab) <= 1e-13 * abs(tab)


def pin_aux_rotation(O):
    """B^P -> sum_Q O_PQ B^Q with O orthogonal: (ia|jb) is unchanged, so E,
    e_ij, P_ij, P_ab are invariant and Gamma rotates the same way."""
    B, eo, ev = tiny_inputs(4, 5, 6, 61)
    Q, _ = np.linalg.qr(np.random.default_rng(62).standard_normal((6, 6)))
    r0 = O.fragment(B, eo, ev)
    r1 = O.fragment(B @ Q, eo, ev)
    assert abs(r1["E"] - r0["E"]) <= 1e-13 * abs(r0["E"])
    for key in ("e_pair", "P_ij", "P_ab"):
        assert rel(r1[key], r0[key]) <= 1e-12, key
    assert rel(r1["Gamma"], r0["Gamma"] @ Q) <= 1e-12


def pin_global_shift(O):
    """eps -> eps + c for occupied and virtual alike leaves every denominator,
    hence every output, unchanged (c chosen so the shift is exact)."""
    B, eo, ev = tiny_inputs(3, 4, 5, 71)
    eo = np.round(eo * 64) / 64
    ev = np.round(ev * 64) / 64
    r0 = O.fragment(B, eo, ev)
    r1 = O.fragment(B, eo + 4.0, ev + 4.0)
    for key in ("e_pair", "Gamma", "P_ij", "P_ab"):
        assert np.array_equal(r0[key], r1[key]), key


def pin_scaling(O):
    """B -> s B: V scales by s^2, so E and P scale by s^4 and Gamma by s^3."""
    B, eo, ev = tiny_inputs(3, 4, 5, 81)
    s = 2.0
    r0 = O.fragment(B, eo, ev)
    r1 = O.fragment(s * B, eo, ev)
    assert abs(r1["E"] - s ** 4 * r0["E"]) <= 1e-14 * abs(r1["E"])
    assert rel(r1["Gamma"], s ** 3 * r0["Gamma"]) <= 1e-14
    assert rel(r1["P_ij"], s ** 4 * r0["P_ij"]) <= 1e-14
    assert rel(r1["P_ab"], s ** 4 * r0["P_ab"]) <= 1e-14


def pin_zero_padding(O):
    """Extra auxiliary functions, virtuals or occupied orbitals whose B is
    zero contribute nothing: E unchanged, padded outputs zero."""
    B, eo, ev = tiny_inputs(3, 4, 5, 91)
    r0 = O.fragment(B, eo, ev)
    Ba = np.concatenate([B, np.zeros((3, 4, 2))], axis=2)
    ra = O.fragment(Ba, eo, ev)
    assert ra["E"] == r0["E"] and rel(ra["Gamma"][:, :, :5], r0["Gamma"]) <= 1e-15
    assert np.all(ra["Gamma"][:, :, 5:] == 0)
    Bv = np.concatenate([B, np.zeros((3, 2, 5))], axis=1)
    rv = O.fragment(Bv, eo, np.concatenate([ev, [6.0, 7.5]]))
    assert abs(rv["E"] - r0["E"]) <= 1e-15 * abs(r0["E"])
    assert rel(rv["P_ab"][:4, :4], r0["P_ab"]) <= 1e-14 and np.all(rv["P_ab"][4:, :] == 0)
    Bo = np.concatenate([np.zeros((1, 4, 5)), B], axis=0)
    ro = O.fragment(Bo, np.concatenate([[-30.0], eo]), ev)
    assert abs(ro["E"] - r0["E"]) <= 1e-15 * abs(r0["E"])
    assert rel(ro["P_ij"][1:, 1:], r0["P_ij"]) <= 1e-14 and np.all(ro["P_ij"][0, :] == 0)


def pin_permutation(O):
    """Relabelling occupied (or virtual) orbitals together with their
    energies permutes the outputs the same way."""
    B, eo, ev = tiny_inputs(4, 5, 3, 101)
    r0 = O.fragment(B, eo, ev)
    po = np.array([2, 0, 3, 1])
    pv = np.array([4, 1, 0, 3, 2])
    r1 = O.fragment(B[po][:, pv], eo[po], ev[pv])
    assert rel(r1["e_pair"], r0["e_pair"][np.ix_(po, po)]) <= 1e-13
    assert rel(r1["Gamma"], r0["Gamma"][po][:, pv]) <= 1e-13
    assert rel(r1["P_ij"], r0["P_ij"][np.ix_(po, po)]) <= 1e-13
    assert rel(r1["P_ab"], r0["P_ab"][np.ix_(pv, pv)]) <= 1e-13


def pin_sampled_entry_points(O):
    """The single-output functions (pair_energy, gamma_row, gamma_rows,
    p_ab_element, p_ij_element) agree with brute force."""
    B, eo, ev = tiny_inputs(3, 4, 5, 111)
    bf = brute_force(B, eo, ev)
    for i in range(3):
        for j in range(3):
            assert abs(O.pair_energy(B, eo, ev, i, j) - bf["e_pair"][i, j]) <= 1e-13 * abs(bf["e_pair"][i, j])
            assert abs(O.p_ij_element(B, eo, ev, i, j) - bf["P_ij"][i, j]) <= 1e-12 * abs(bf["P_ij"]).max()
    for i in range(3):
        for a in range(4):
            assert rel(O.gamma_row(B, eo, ev, i, a), bf["Gamma"][i, a]) <= 1e-12
        assert rel(O.gamma_rows(B, eo, ev, i, [3, 0, 2]), bf["Gamma"][i, [3, 0, 2]]) <= 1e-12
    for a in range(4):
        for b in range(4):
            assert abs(O.p_ab_element(B, eo, ev, a, b) - bf["P_ab"][a, b]) <= 1e-12 * abs(bf["P_ab"]).max()


def pin_exact_sum(O):
    """E_hi + E_lo is the exact sum: values whose float sum loses digits."""
    vals = np.array([1e16, 1.0, -1e16, 3.0, 1e-3])
    hi, lo = O.exact_sum(vals)
    assert hi == 4.001 and abs(lo) < 1e-15
    vals = np.array([2.0 ** 60, 1.0, 1.0])
    hi, lo = O.exact_sum(vals)
    assert hi == 2.0 ** 60 and lo == 2.0


def pin_gamma_metric_is_three_centre_derivative(O):
    """With B = B3 M (B[..., P] = sum_Q B3[..., Q] M[Q, P]; in the paper M =
    J^{-1/2} and B3 the three-centre integrals), the chain rule and
    dE/dB = 4 Gamma give dE/dB3 = 4 gamma_metric(Gamma, M), by complex step
    of the energy.  M is not symmetric, so a transposed metric fails."""
    h = 1e-30
    B3, eo, ev = tiny_inputs(2, 3, 4, 21)
    M = np.random.default_rng(22).standard_normal((4, 4))
    want = 4.0 * O.gamma_metric(O.fragment(B3 @ M, eo, ev, density=False)["Gamma"], M)
    got = np.zeros_like(B3)
    for idx in np.ndindex(B3.shape):
        Bc = B3.astype(np.complex128)
        Bc[idx] += 1j * h
        got[idx] = _complex_E(O, Bc @ M, eo, ev).imag / h
    assert rel(got, want) <= 1e-12, rel(got, want)


ALL_PINS = [pin_brute_force, pin_closed_form_single_pair, pin_equal_energies, pin_dE_dB_is_4_gamma,
            pin_dE_deps_is_2_diagP, pin_symmetry_and_sign, pin_aux_rotation, pin_global_shift,
            pin_scaling, pin_zero_padding, pin_permutation, pin_sampled_entry_points, pin_exact_sum,
            pin_gamma_metric_is_three_centre_derivative]


def pin_skip_all_pairs_of_an_orbital_deletes_it(O):
    """Screening out every pair {i, j} that contains occupied orbital i (the
    diagonal pair included) leaves exactly the fragment without orbital i:
    E and the other e_jk, Gamma rows and P_ij entries not involving i, and
    P_ab equal the oracle run on B and eps_occ with orbital i removed; row i
    of Gamma and row and column i of e_pair and P_ij are zero.  A mask that
    marks only row i names the same unordered pairs as one that marks row
    and column i."""
    nocc, nvir, naux = 4, 3, 5
    B, eo, ev = tiny_inputs(nocc, nvir, naux, 21)
    for i in (0, 2, nocc - 1):
        keep = [k for k in range(nocc) if k != i]
        red = O.fragment(B[keep], eo[keep], ev)
        for half in (False, True):
            skip = np.zeros((nocc, nocc), dtype=np.uint8)
            skip[i, :] = 1          # row i alone names every pair {i, j}
            if not half:
                skip[:, i] = 1
            got = O.fragment(B, eo, ev, skip=skip)
            assert abs(got["E_hi"] - red["E_hi"]) <= RTOL * abs(red["E_hi"])
            assert rel(got["e_pair"][np.ix_(keep, keep)], red["e_pair"]) <= RTOL
            assert np.all(got["e_pair"][i, :] == 0) and np.all(got["e_pair"][:, i] == 0)
            assert rel(got["Gamma"][keep], red["Gamma"]) <= RTOL
            assert np.all(got["Gamma"][i] == 0)
            assert rel(got["P_ij"][np.ix_(keep, keep)], red["P_ij"]) <= RTOL
            assert np.all(got["P_ij"][i, :] == 0) and np.all(got["P_ij"][:, i] == 0)
            assert rel(got["P_ab"], red["P_ab"]) <= RTOL


def pin_skip_nothing_is_the_full_result(O):
    """An all-zero mask screens nothing out: every output is the unscreened
    one, bit for bit; a mask over one pair zeroes exactly e_ij and e_ji."""
    B, eo, ev = tiny_inputs(3, 4, 5, 22)
    full = O.fragment(B, eo, ev)
    got = O.fragment(B, eo, ev, skip=np.zeros((3, 3), dtype=np.uint8))
    for key in ("e_pair", "Gamma", "P_ij", "P_ab"):
        assert np.array_equal(got[key], full[key])
    skip = np.zeros((3, 3), dtype=np.uint8)
    skip[2, 0] = 1
    one = O.fragment(B, eo, ev, skip=skip)
    ref = full["e_pair"].copy()
    ref[0, 2] = ref[2, 0] = 0.0
    assert np.array_equal(one["e_pair"], ref)


ALL_PINS.extend([pin_skip_all_pairs_of_an_orbital_deletes_it, pin_skip_nothing_is_the_full_result])


def pin_gamma_ao_is_ao_derivative(O):
    """With the MO transform of the paper, B^P_ia = sum_mn C_im C_an B^P_mn
    (B[i, a, P] = sum_mn C_occ[i, m] C_vir[a, n] B_ao[m, n, P]), the chain
    rule and dE/dB = 4 Gamma give dE/dB_ao = 4 gamma_ao(Gamma, C_occ, C_vir),
    checked by complex step of the energy for every element of B_ao.  The
    coefficient matrices are rectangular and different, so a transposed or
    swapped one fails."""
    h = 1e-30
    nocc, nvir, nao, naux = 2, 3, 4, 3
    rng = np.random.default_rng(31)
    C_occ = rng.standard_normal((nocc, nao))
    C_vir = rng.standard_normal((nvir, nao))
    B_ao = 0.3 * rng.standard_normal((nao, nao, naux))
    _, eo, ev = tiny_inputs(nocc, nvir, naux, 32)

    def mo(Bao):
        return np.einsum("im,an,mnP->iaP", C_occ, C_vir, Bao)

    want = 4.0 * O.gamma_ao(O.fragment(mo(B_ao), eo, ev, density=False)["Gamma"], C_occ, C_vir)
    got = np.zeros_like(B_ao)
    for idx in np.ndindex(B_ao.shape):
        Bc = B_ao.astype(np.complex128)
        Bc[idx] += 1j * h
        got[idx] = _complex_E(O, mo(Bc), eo, ev).imag / h
    assert rel(got, want) <= 1e-12, rel(got, want)


def _three_centre_system(seed, nocc=2, nvir=3, naux=4):
    """Three-centre MO integrals I[Q][p][q] (symmetric in p, q over all
    nocc + nvir orbitals, occupied first), a non-symmetric metric factor M,
    and orbital energies."""
    rng = np.random.default_rng(seed)
    nmo = nocc + nvir
    I = 0.3 * rng.standard_normal((naux, nmo, nmo))
    I = I + I.transpose(0, 2, 1)
    M = rng.standard_normal((naux, naux))
    _, eo, ev = tiny_inputs(nocc, nvir, naux, seed + 1)
    return I, M, eo, ev


def pin_l_terms_are_orbital_rotation_derivatives(O):
    """L'_iq and L'' _aq are a quarter of the derivatives of E with respect
    to mixing orbital q into occupied orbital i, or into virtual orbital a,
    in the three-centre integrals (P|ia) from which B = (P|ia) J^{-1/2} is
    formed: with B3[i, a, Q] = (Q|ia) and B = B3 M,
      d/dt E(B3[i, :, :] += t (.|q.)) = 4 L'_iq,
      d/dt E(B3[:, a, :] += t (.|.q)) = 4 L''_aq,
    where Gamma is gamma_metric(Gamma~, M), the Appendix's Gamma with its
    metric contraction (complex step, every i, a and q)."""
    h = 1e-30
    nocc, nvir, naux = 2, 3, 4
    I, M, eo, ev = _three_centre_system(41, nocc, nvir, naux)
    nmo = nocc + nvir
    B3 = np.transpose(I[:, :nocc, nocc:], (1, 2, 0)).copy()     # B3[i, a, Q] = (Q|ia)
    I_qa = np.transpose(I[:, :, nocc:], (1, 2, 0)).copy()       # I_qa[q, a, Q] = (Q|qa)
    I_iq = np.transpose(I[:, :nocc, :], (1, 2, 0)).copy()       # I_iq[i, q, Q] = (Q|iq)
    G = O.gamma_metric(O.fragment(B3 @ M, eo, ev, density=False)["Gamma"], M)
    L1 = O.l_prime(G, I_qa)
    L2 = O.l_dprime(G, I_iq)
    assert L1.shape == (nocc, nmo) and L2.shape == (nvir, nmo)
    for i in range(nocc):
        for q in range(nmo):
            Bc = B3.astype(np.complex128)
            Bc[i] += 1j * h * I_qa[q]
            d = _complex_E(O, Bc @ M, eo, ev).imag / h
            assert abs(d - 4.0 * L1[i, q]) <= 1e-12 * max(1.0, abs(d)), (i, q, d, 4.0 * L1[i, q])
    for a in range(nvir):
        for q in range(nmo):
            Bc = B3.astype(np.complex128)
            Bc[:, a, :] += 1j * h * I_iq[:, q, :]
            d = _complex_E(O, Bc @ M, eo, ev).imag / h
            assert abs(d - 4.0 * L2[a, q]) <= 1e-12 * max(1.0, abs(d)), (a, q, d, 4.0 * L2[a, q])


ALL_PINS.extend([pin_gamma_ao_is_ao_derivative, pin_l_terms_are_orbital_rotation_derivatives])


def _response_inputs(seed, nocc=2, nvir=3, naux=4, scale=0.1):
    """Full three-index factor Bf [nmo][nmo][naux] (symmetric in the MO pair),
    orbital energies, symmetric D_ij and D_ab blocks, and L' / L'' terms."""
    rng = np.random.default_rng(seed)
    nmo = nocc + nvir
    Bf = scale * rng.standard_normal((nmo, nmo, naux))
    Bf = 0.5 * (Bf + Bf.transpose(1, 0, 2))
    _, eo, ev = tiny_inputs(nocc, nvir, naux, seed + 1)
    D_oo = rng.standard_normal((nocc, nocc))
    D_vv = rng.standard_normal((nvir, nvir))
    L1 = rng.standard_normal((nocc, nmo))
    L2 = rng.standard_normal((nvir, nmo))
    return Bf, eo, ev, D_oo + D_oo.T, D_vv + D_vv.T, L1, L2


def _solve_gauss(A, b):
    """Gauss-Jordan elimination with partial pivoting, pure Python."""
    n = len(b)
    M = [list(map(float, A[r])) + [float(b[r])] for r in range(n)]
    for c in range(n):
        piv = max(range(c, n), key=lambda r: abs(M[r][c]))
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[r][n] / M[r][r] for r in range(n)]


def pin_zvector_brute_force(O):
    """The antisymmetrised-integral term and the Z-vector solution against
    pure-Python loops over the Appendix's index forms: G_pq^rs = 2 (pq|rs) -
    (ps|rq), the right-hand side L''_ai - L'_ia - sum_pq G_ai^pq Dbar_pq, the
    operator (eps_a - eps_i)/2 D_ai + sum_bj G_ai^bj D_bj, solved by
    Gauss-Jordan elimination."""
    nocc, nvir, naux = 2, 3, 4
    Bf, eo, ev, D_oo, D_vv, L1, L2 = _response_inputs(51, nocc, nvir, naux)
    nmo = nocc + nvir
    eri = lambda p, q, r, t: sum(Bf[p, q, P] * Bf[r, t, P] for P in range(naux))
    G = {(p, q, r, t): 2.0 * eri(p, q, r, t) - eri(p, t, r, q)
         for p in range(nmo) for q in range(nmo) for r in range(nmo) for t in range(nmo)}
    D = np.zeros((nmo, nmo))
    D[:nocc, :nocc], D[nocc:, nocc:] = D_oo, D_vv
    D[nocc:, :nocc] = np.arange(nvir * nocc).reshape(nvir, nocc) * 0.1   # an ov block for the term alone
    F = np.array([[sum(G[p, q, r, t] * D[r, t] for r in range(nmo) for t in range(nmo)) for q in range(nmo)]
                  for p in range(nmo)])
    assert rel(O.antisym_term(Bf, D), F) <= 1e-12
    Dbar = np.zeros((nmo, nmo))
    Dbar[:nocc, :nocc], Dbar[nocc:, nocc:] = D_oo, D_vv
    rows = [(a, i) for a in range(nvir) for i in range(nocc)]
    rhs = [L2[a, i] - L1[i, nocc + a] - sum(G[nocc + a, i, p, q] * Dbar[p, q] for p in range(nmo) for q in range(nmo))
           for a, i in rows]
    A = [[(ev[a] - eo[i]) / 2.0 * (a == b and i == j) + G[nocc + a, i, nocc + b, j] for b, j in rows] for a, i in rows]
    want = np.array(_solve_gauss(A, rhs)).reshape(nvir, nocc)
    assert rel(O.zvector(Bf, eo, ev, D_oo, D_vv, L1, L2), want) <= 1e-11


def pin_zvector_single_pair(O):
    """nocc = nvir = 1: G_ai^ai = 2 (ai|ai) - (ai|ai) = (ai|ai), so
    D_ai = (L''_ai - L'_ia - sum_pq G_ai^pq Dbar_pq) / ((eps_a - eps_i)/2 + (ai|ai)),
    with sum_pq G_ai^pq Dbar_pq = [2 (ai|ii) - (ai|ii)] D_ii + [2 (ai|aa) - (aa|ai)] D_aa."""
    Bf, eo, ev, D_oo, D_vv, L1, L2 = _response_inputs(52, 1, 1, 5)
    aiai = float(Bf[1, 0] @ Bf[1, 0])
    aiii = float(Bf[1, 0] @ Bf[0, 0])
    aiaa = float(Bf[1, 0] @ Bf[1, 1])
    rhs = L2[0, 0] - L1[0, 1] - (aiii * D_oo[0, 0] + aiaa * D_vv[0, 0])
    want = rhs / ((ev[0] - eo[0]) / 2.0 + aiai)
    got = O.zvector(Bf, eo, ev, D_oo, D_vv, L1, L2)
    assert got.shape == (1, 1) and abs(got[0, 0] - want) <= 1e-13 * max(1.0, abs(want))


def pin_energy_weighted_density_hf_limit(O):
    """With no MP2 density and no L terms, W is the HF energy-weighted
    density: eps_i on the occupied diagonal, zero elsewhere (the MO form of
    sum_i eps_i C_imu C_inu).  With them, the occupied rows carry
    sum_rs G_iq^rs D^MP2_rs + L'_iq and the virtual rows L''_aq on top of
    (eps_p + eps_q)/2 D_pq, checked against pure-Python loops."""
    nocc, nvir, naux = 2, 3, 4
    Bf, eo, ev, D_oo, D_vv, L1, L2 = _response_inputs(53, nocc, nvir, naux)
    nmo = nocc + nvir
    z = np.zeros
    W0 = O.energy_weighted_density(Bf, eo, ev, z((nocc, nocc)), z((nvir, nvir)), z((nvir, nocc)),
                                   z((nocc, nmo)), z((nvir, nmo)))
    want = np.zeros((nmo, nmo))
    want[:nocc, :nocc] = np.diag(eo)
    assert rel(W0, want) <= 1e-15
    D_vo = np.random.default_rng(54).standard_normal((nvir, nocc))
    W = O.energy_weighted_density(Bf, eo, ev, D_oo, D_vv, D_vo, L1, L2)
    eps = list(eo) + list(ev)
    Dm = np.zeros((nmo, nmo))
    Dm[:nocc, :nocc], Dm[nocc:, nocc:], Dm[nocc:, :nocc], Dm[:nocc, nocc:] = D_oo, D_vv, D_vo, D_vo.T
    eri = lambda p, q, r, t: sum(Bf[p, q, P] * Bf[r, t, P] for P in range(naux))
    ref = np.zeros((nmo, nmo))
    for p in range(nmo):
        for q in range(nmo):
            d = Dm[p, q] + (1.0 if (p == q and p < nocc) else 0.0)
            w = (eps[p] + eps[q]) / 2.0 * d
            if p < nocc:
                w += sum((2.0 * eri(p, q, r, t) - eri(p, t, r, q)) * Dm[r, t] for r in range(nmo) for t in range(nmo))
                w += L1[p, q]
            else:
                w += L2[p - nocc, q]
            ref[p, q] = w
    assert rel(W, ref) <= 1e-12


ALL_PINS.extend([pin_zvector_brute_force, pin_zvector_single_pair, pin_energy_weighted_density_hf_limit])

