"""CPU oracle for the closed-shell RI-MP2 fragment kernel.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this module; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path.

It is a plain, slow, FP64 statement of what the kernel computes, following the
paper (arXiv 2410.21888):

* RI factorisation of the MO integrals, (ia|jb) = sum_P B^P_ia B^P_jb
  (Sec. "Resolution-of-the-Identity HF and MP2", Eq. MP2_ints).
* Amplitudes X_ij^ab = (ia|jb) / (eps_i + eps_j - eps_a - eps_b) (Appendix,
  definition of the RI-MP2 amplitudes; the denominator is the textual
  expansion of the paper's macros).
* Gamma^P_ia = sum_jb (2 X_ij^ab - X_ij^ba) B^P_jb (Appendix, definition of
  Gamma, taken before the J^{-1/2} back-contraction).
* P_ij = -sum_abk (2 X_ik^ab - X_ki^ab) X_jk^ab and
  P_ab = sum_ijc (2 X_ij^ac - X_ij^ca) X_ij^bc (Appendix, occupied-occupied and
  virtual-virtual blocks of D^MP2).
* E_MP2 = sum_ij sum_ab (ia|jb) [2 (ia|jb) - (ib|ja)] / D_ij^ab, the canonical
  closed-shell RI-MP2 energy named in Sec. "Molecular Fragmentation"
  (Eq. efrag).  The paper does not print it; it is the unique energy whose
  derivative with respect to B is 4 Gamma, the factor in the Appendix's
  three-centre gradient coefficient Z = 4 Gamma + ...

Closed shell, no frozen core (Sec. "Background": restricted closed-shell HF
and MP2 without the frozen-core approximation): every occupied orbital is
correlated.

Notation: B has shape [nocc][nvir][naux] (P fastest); B_i = B[i] is nvir x naux.
V_ij = B_i B_j^T, D_ij[a, b] = eps_i + eps_j - eps_a - eps_b, X_ij = V_ij / D_ij,
T_ij = 2 X_ij - X_ij^T (so T_ij[a, b] = 2 X_ij^ab - X_ij^ba = 2 X_ij^ab - X_ji^ab).

Every function works for real float64 inputs and, for the complex-step
derivative tests, for complex128 inputs (no conjugation anywhere).

Parity status of each function (how it is pinned) is listed in the test
module ``tests/test_oracle_pins.py``; every function here is pinned.
"""
from __future__ import annotations

import math

import numpy as np


def pair_integrals(B_i: np.ndarray, B_j: np.ndarray) -> np.ndarray:
    """V_ij[a, b] = (ia|jb)_RI = sum_P B^P_ia B^P_jb (Eq. MP2_ints)."""
    return B_i @ B_j.T


def denominators(e_i, e_j, eps_vir: np.ndarray) -> np.ndarray:
    """D_ij[a, b] = eps_i + eps_j - eps_a - eps_b (Appendix, amplitude
    denominator, macros expanded as written)."""
    return (e_i + e_j) - eps_vir[:, None] - eps_vir[None, :]


def amplitudes(V_ij: np.ndarray, D_ij: np.ndarray) -> np.ndarray:
    """X_ij^ab = (ia|jb) / D_ij^ab (Appendix, RI-MP2 amplitudes)."""
    return V_ij / D_ij


def combination(X_ij: np.ndarray) -> np.ndarray:
    """T_ij^ab = 2 X_ij^ab - X_ij^ba, the combination that appears in Gamma and
    in both density blocks (Appendix)."""
    return 2.0 * X_ij - X_ij.T


def pair_quantities(B, eps_occ, eps_vir, i: int, j: int):
    """(V_ij, X_ij, T_ij) for one ordered occupied pair."""
    V = pair_integrals(B[i], B[j])
    X = amplitudes(V, denominators(eps_occ[i], eps_occ[j], eps_vir))
    return V, X, combination(X)


def pair_energy(B, eps_occ, eps_vir, i: int, j: int):
    """e_ij = sum_ab (ia|jb) [2 (ia|jb) - (ib|ja)] / D_ij^ab = sum_ab T_ij V_ij."""
    V, X, T = pair_quantities(B, eps_occ, eps_vir, i, j)
    return np.sum(T * V)


def exact_sum(values) -> tuple[float, float]:
    """Correctly rounded sum of float64 values, plus the rounded remainder, so
    that hi + lo represents the exact sum to about 2^-106 relative."""
    vals = [float(v) for v in np.ravel(values)]
    hi = math.fsum(vals)
    lo = math.fsum(vals + [-hi])
    return hi, lo


def fragment(B, eps_occ, eps_vir, gamma: bool = True, density: bool = True, slabs=None, skip=None) -> dict:
    """All outputs of the fragment kernel.

    Returns a dict with
      e_pair [nocc][nocc]  e_ij for every ordered pair (e_ij = e_ji)
      E_hi, E_lo           E_MP2 = sum_ij e_ij, exactly rounded (real inputs)
      E                    plain sum (complex inputs)
      Gamma [nocc][nvir][naux], P_ij [nocc][nocc], P_ab [nvir][nvir]
    The loop runs over the occupied index k of the first orbital of each pair;
    for each k it forms V_kj, X_kj, T_kj for all j as plain matrices.
    ``slabs`` (an iterable of k) restricts the loop to those k: then e_pair
    rows and Gamma rows k are complete, the other rows stay zero, P_ij and P_ab
    hold only those slabs' contributions and E sums the computed rows.
    ``skip`` ([nocc][nocc], or None) screens occupied pairs out: a nonzero
    skip[k, j] or skip[j, k] removes the unordered pair {k, j}, which then has
    no amplitudes (X_kj = T_kj = 0 in both orders) and e_kj = 0.  This is the
    pair screening the learned model drives; the mask names unordered pairs.
    """
    B = np.asarray(B)
    nocc, nvir, naux = B.shape
    dt = np.result_type(B.dtype, np.asarray(eps_occ).dtype, np.asarray(eps_vir).dtype, np.float64)
    e_pair = np.zeros((nocc, nocc), dtype=dt)
    Gamma = np.zeros((nocc, nvir, naux), dtype=dt) if gamma else None
    P_ij = np.zeros((nocc, nocc), dtype=dt) if density else None
    P_ab = np.zeros((nvir, nvir), dtype=dt) if density else None
    for k in (range(nocc) if slabs is None else slabs):
        X_k = np.zeros((nocc, nvir, nvir), dtype=dt)
        T_k = np.zeros((nocc, nvir, nvir), dtype=dt)
        for j in range(nocc):
            if skip is not None and (skip[k][j] or skip[j][k]):
                continue            # screened out: X_kj = T_kj = 0, e_kj = 0
            V, X, T = pair_quantities(B, eps_occ, eps_vir, k, j)
            X_k[j], T_k[j] = X, T
            e_pair[k, j] = np.sum(T * V)
            if gamma:
                # Gamma_k[a, P] += sum_b T_kj[a, b] B_j[b, P]
                Gamma[k] += T @ B[j]
            if density:
                # P_ab[a, b] += sum_c T_kj[a, c] X_kj[b, c]
                P_ab += T @ X.T
        if density:
            # The paper's P_ij = -sum_k <T_ik, X_jk>_F.  Since T_ki = T_ik^T,
            # X_kj = X_jk^T and a Frobenius product is unchanged when both
            # factors are transposed, this equals -sum_k <T_ki, X_kj>_F, which
            # is what slab k holds: P_ij[i, j] -= sum_ab T_ki[a, b] X_kj[a, b].
            P_ij -= T_k.reshape(nocc, -1) @ X_k.reshape(nocc, -1).T
    out = {"e_pair": e_pair, "Gamma": Gamma, "P_ij": P_ij, "P_ab": P_ab}
    if np.iscomplexobj(e_pair):
        out["E"] = np.sum(e_pair)
    else:
        out["E_hi"], out["E_lo"] = exact_sum(e_pair)
        out["E"] = out["E_hi"]
    return out


# ---------------------------------------------------------------------------
# Single outputs at any size, for sampled checks of large problems.  Each
# needs only the rows of B named in its docstring, so a caller may pass a
# lazily generated B (anything indexable by occupied index).
# ---------------------------------------------------------------------------

def gamma_row(B, eps_occ, eps_vir, i: int, a: int) -> np.ndarray:
    """Gamma[i, a, :] = sum_j sum_b T_ij[a, b] B_j[b, :].

    Needs row a and column a of every V_ij: V_ij[a, :] = B_i[a] B_j^T and
    V_ij[:, a] = B_i B_j[a]."""
    nocc = len(eps_occ)
    out = 0.0
    for j in range(nocc):
        Bj = B[j]
        row = Bj @ B[i][a]          # V_ij[a, b] over b
        col = B[i] @ Bj[a]          # V_ij[b, a] over b
        D_row = denominators(eps_occ[i], eps_occ[j], eps_vir)[a]
        T_row = 2.0 * row / D_row - col / D_row   # D_ij is symmetric in (a, b)
        out = out + T_row @ Bj
    return out


def gamma_rows(B, eps_occ, eps_vir, i: int, rows) -> np.ndarray:
    """Gamma[i, a, :] for every a in ``rows`` ([len(rows)][naux]), as
    gamma_row computes one, with a single pass over the rows of B."""
    rows = np.asarray(list(rows), dtype=np.int64)
    nocc = len(eps_occ)
    out = 0.0
    for j in range(nocc):
        Bj = B[j]
        V_row = B[i][rows] @ Bj.T   # V_ij[a, b] for a in rows
        V_col = Bj[rows] @ B[i].T   # V_ij[b, a] for a in rows (indexed [a][b])
        D = denominators(eps_occ[i], eps_occ[j], eps_vir)[rows]
        T = 2.0 * V_row / D - V_col / D
        out = out + T @ Bj
    return out


def p_ab_element(B, eps_occ, eps_vir, a: int, b: int):
    """P_ab[a, b] = sum_ij sum_c T_ij[a, c] X_ij[b, c]."""
    nocc = len(eps_occ)
    s = 0.0
    for i in range(nocc):
        for j in range(nocc):
            Bi, Bj = B[i], B[j]
            D = denominators(eps_occ[i], eps_occ[j], eps_vir)
            Va_row = Bj @ Bi[a]     # V_ij[a, c]
            Va_col = Bi @ Bj[a]     # V_ij[c, a]
            Vb_row = Bj @ Bi[b]     # V_ij[b, c]
            T_a = (2.0 * Va_row - Va_col) / D[a]
            X_b = Vb_row / D[b]
            s = s + T_a @ X_b
    return s


def p_ij_element(B, eps_occ, eps_vir, i: int, j: int):
    """P_ij[i, j] = -sum_k <T_ik, X_jk>_F = -sum_k sum_ab T_ki[a, b] X_kj[a, b]
    (both factors transposed, see ``fragment``)."""
    nocc = len(eps_occ)
    s = 0.0
    for k in range(nocc):
        _, _, T = pair_quantities(B, eps_occ, eps_vir, k, i)
        _, X, _ = pair_quantities(B, eps_occ, eps_vir, k, j)
        s = s + np.sum(T * X)
    return -s


def gamma_metric(Gamma, Jm):
    """The Appendix's Gamma^P_ia = sum_Q Gamma~^Q_ia J^{-1/2}_PQ, from the
    fragment kernel's Gamma~ (taken before this contraction; see the module
    header): out[i, a, P] = sum_Q Gamma[i, a, Q] Jm[P, Q]."""
    return Gamma @ Jm.T


# ---------------------------------------------------------------------------
# Adjacent gradient steps (Appendix): the AO back-transform of Gamma and the
# L' and L'' terms of the energy-weighted density matrix.
# ---------------------------------------------------------------------------

def gamma_ao(Gamma, C_occ, C_vir):
    """Gamma^P_ia back-transformed to the AO basis (Appendix, after the
    definition of Gamma): Gamma^P_mn = sum_ia C_im Gamma^P_ia C_an, with the
    MO coefficients stored C_occ[i][m] and C_vir[a][n] (the paper's C_imu):
    out[m, n, P] = sum_i sum_a C_occ[i, m] Gamma[i, a, P] C_vir[a, n]."""
    return np.einsum("im,iaP,an->mnP", C_occ, Gamma, C_vir)


def l_prime(Gamma, I_qa):
    """L'_iq = sum_aP Gamma^P_ia (P|qa) (Appendix, energy-weighted density),
    with I_qa[q, a, P] = (P|qa) for every molecular orbital q."""
    return np.einsum("iaP,qaP->iq", Gamma, I_qa)


def l_dprime(Gamma, I_iq):
    """L''_aq = sum_iP Gamma^P_ia (P|iq) (Appendix, energy-weighted density),
    with I_iq[i, q, P] = (P|iq) for every molecular orbital q."""
    return np.einsum("iaP,iqP->aq", Gamma, I_iq)


# ---------------------------------------------------------------------------
# Orbital-response steps (Appendix): the antisymmetrised-integral term, the
# Z-vector equation for the occupied-virtual block of the MP2 density, and the
# energy-weighted density matrix.  Bf[p, q, P] is the three-index factor over
# every pair of molecular orbitals (occupied first, symmetric in p and q); its
# occupied-virtual block Bf[i, nocc + a] is the fragment kernel's B[i, a].
# ---------------------------------------------------------------------------

def antisym_term(Bf, D):
    """F[p, q] = sum_rs G_pq^rs D_rs, with the Appendix's antisymmetrised
    integrals G_pq^rs = 2 (pq|rs) - (ps|rq) and (pq|rs) = sum_P Bf[p, q, P]
    Bf[r, s, P] (RI)."""
    coulomb = np.einsum("pqP,rsP,rs->pq", Bf, Bf, D)
    exchange = np.einsum("psP,rqP,rs->pq", Bf, Bf, D)
    return 2.0 * coulomb - exchange


def zvector(Bf, eps_occ, eps_vir, D_oo, D_vv, L1, L2):
    """The occupied-virtual block D_ai of the MP2 density from the Appendix's
    Z-vector equation,

      L''_ai - L'_ia - sum_pq G_ai^pq Dbar_pq
          = (eps_a - eps_i)/2 D_ai + sum_bj G_ai^bj D_bj,

    with Dbar = D_ij (+) D_ab (zero occupied-virtual blocks), L1 = L' [nocc][nmo]
    and L2 = L'' [nvir][nmo] (column q an MO index).  The left side is the
    right-hand vector; the right side's operator is assembled as the matrix
    A[(a,i), (b,j)] = delta_ab delta_ij (eps_a - eps_i)/2 + 2 (ai|bj) - (aj|bi)
    and the system is solved directly.  Returns D_ai as [nvir][nocc]."""
    nocc, nvir = len(eps_occ), len(eps_vir)
    nmo = nocc + nvir
    Dbar = np.zeros((nmo, nmo), dtype=np.result_type(Bf, D_oo, D_vv))
    Dbar[:nocc, :nocc] = D_oo
    Dbar[nocc:, nocc:] = D_vv
    rhs = L2[:, :nocc] - L1[:, nocc:].T - antisym_term(Bf, Dbar)[nocc:, :nocc]
    Bvo = Bf[nocc:, :nocc]                                    # [a][i][P]
    coulomb = np.einsum("aiP,bjP->aibj", Bvo, Bvo)            # (ai|bj)
    exchange = np.einsum("ajP,biP->aibj", Bvo, Bvo)           # (aj|bi)
    A = 2.0 * coulomb - exchange
    nov = nvir * nocc
    A = A.reshape(nov, nov) + np.diag(((eps_vir[:, None] - eps_occ[None, :]) / 2.0).ravel())
    return np.linalg.solve(A, rhs.ravel()).reshape(nvir, nocc)


def energy_weighted_density(Bf, eps_occ, eps_vir, D_oo, D_vv, D_vo, L1, L2):
    """The Appendix's energy-weighted density matrix W [nmo][nmo], read as the
    sum of its four printed pieces over the parts of the (p, q) domain they
    fill:
      W_pq  = (eps_p + eps_q)/2 D_pq                      every p, q
            + sum_rs G_pq^rs D^MP2_rs + L'_pq              occupied rows p = i
            + L''_pq                                       virtual rows p = a
    with D = D^HF + D^MP2, D^HF the identity on the occupied block (the MO
    form of sum_i C_imu C_inu), and D^MP2 = D_ij (+) D_ab (+) D_ai (+) D_ia
    (D_ia = D_ai)."""
    nocc, nvir = len(eps_occ), len(eps_vir)
    nmo = nocc + nvir
    eps = np.concatenate([eps_occ, eps_vir])
    Dm = np.zeros((nmo, nmo), dtype=np.result_type(Bf, D_oo, D_vv, D_vo))
    Dm[:nocc, :nocc] = D_oo
    Dm[nocc:, nocc:] = D_vv
    Dm[nocc:, :nocc] = D_vo
    Dm[:nocc, nocc:] = D_vo.T
    D = Dm.copy()
    D[:nocc, :nocc] += np.eye(nocc)
    W = (eps[:, None] + eps[None, :]) / 2.0 * D
    W[:nocc] += antisym_term(Bf, Dm)[:nocc] + L1
    W[nocc:] += L2
    return W

