"""Planted mistakes in the oracle must each fail at least one pin.

Each mutant is the oracle's own source with one plausible mistake planted
(a dropped term, a wrong sign, a wrong index, a transposed operand, a misread
denominator), loaded as a separate module on the CPU.  The real oracle is
never modified.
"""
import importlib.util
import os
import types

import pytest

import pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "rimp2_oracle.py")

MUTANTS = [
    ("exchange term dropped", "return 2.0 * X_ij - X_ij.T", "return 2.0 * X_ij"),
    ("exchange sign flipped", "return 2.0 * X_ij - X_ij.T", "return 2.0 * X_ij + X_ij.T"),
    ("transpose missing", "return 2.0 * X_ij - X_ij.T", "return 2.0 * X_ij - X_ij"),
    ("denominator read as (ei+ej)-(ea-eb)", "return (e_i + e_j) - eps_vir[:, None] - eps_vir[None, :]",
     "return (e_i + e_j) - (eps_vir[:, None] - eps_vir[None, :])"),
    ("denominator sign", "return (e_i + e_j) - eps_vir[:, None] - eps_vir[None, :]",
     "return eps_vir[:, None] + eps_vir[None, :] - (e_i + e_j)"),
    ("pair integrals operands swapped", "return B_i @ B_j.T", "return B_j @ B_i.T"),
    ("pair integrals wrong index", "V = pair_integrals(B[i], B[j])", "V = pair_integrals(B[i], B[i])"),
    ("denominator wrong index", "denominators(eps_occ[i], eps_occ[j], eps_vir))",
     "denominators(eps_occ[i], eps_occ[i], eps_vir))"),
    ("amplitude multiplies", "return V_ij / D_ij", "return V_ij * D_ij"),
    ("energy uses X for T", "e_pair[k, j] = np.sum(T * V)", "e_pair[k, j] = np.sum(X * V)"),
    ("energy factor 2", "e_pair[k, j] = np.sum(T * V)", "e_pair[k, j] = np.sum(2.0 * T * V)"),
    ("pair loop misses j = 0", "for j in range(nocc):\n            if skip", "for j in range(1, nocc):\n            if skip"),
    ("Gamma uses X for T", "Gamma[k] += T @ B[j]", "Gamma[k] += X @ B[j]"),
    ("Gamma transposed T", "Gamma[k] += T @ B[j]", "Gamma[k] += T.T @ B[j]"),
    ("Gamma wrong B row", "Gamma[k] += T @ B[j]", "Gamma[k] += T @ B[k]"),
    ("P_ab X not transposed", "P_ab += T @ X.T", "P_ab += T @ X"),
    ("P_ab uses V for X", "P_ab += T @ X.T", "P_ab += T @ V.T"),
    ("P_ij sign", "P_ij -= T_k.reshape", "P_ij += T_k.reshape"),
    ("P_ij uses X for T", "P_ij -= T_k.reshape(nocc, -1)", "P_ij -= X_k.reshape(nocc, -1)"),
    ("exact sum drops remainder", "lo = math.fsum(vals + [-hi])", "lo = 0.0"),
    ("gamma_row exchange from row", "T_row = 2.0 * row / D_row - col / D_row", "T_row = 2.0 * row / D_row - row / D_row"),
    ("p_ab_element wrong denominator", "X_b = Vb_row / D[b]", "X_b = Vb_row / D[a]"),
    ("p_ij_element sign", "    return -s\n", "    return s\n"),
    ("gamma_metric transposed", "return Gamma @ Jm.T", "return Gamma @ Jm"),
    ("gamma_metric drops the metric", "return Gamma @ Jm.T", "return Gamma"),
    ("gamma_rows exchange from row", "T = 2.0 * V_row / D - V_col / D", "T = 2.0 * V_row / D - V_row / D"),
    ("gamma_rows wrong exchange index", "V_col = Bj[rows] @ B[i].T", "V_col = B[i][rows] @ Bj.T"),
    ("gamma_ao coefficients swapped", 'np.einsum("im,iaP,an->mnP", C_occ, Gamma, C_vir)',
     'np.einsum("an,iaP,im->mnP", C_occ, Gamma, C_vir)'),
    ("gamma_ao output transposed", 'np.einsum("im,iaP,an->mnP", C_occ, Gamma, C_vir)',
     'np.einsum("im,iaP,an->nmP", C_occ, Gamma, C_vir)'),
    ("l_prime aux index not matched", 'np.einsum("iaP,qaP->iq", Gamma, I_qa)', 'np.einsum("iaP,qaQ->iq", Gamma, I_qa)'),
    ("l_dprime aux index not matched", 'np.einsum("iaP,iqP->aq", Gamma, I_iq)', 'np.einsum("iaP,iqQ->aq", Gamma, I_iq)'),
    ("l_dprime occupied index not matched", 'np.einsum("iaP,iqP->aq", Gamma, I_iq)',
     'np.einsum("iaP,jqP->aq", Gamma, I_iq)'),
    ("antisymmetrised term exchange indices", 'exchange = np.einsum("psP,rqP,rs->pq", Bf, Bf, D)',
     'exchange = np.einsum("pqP,rsP,rs->pq", Bf, Bf, D)'),
    ("Z-vector operator exchange indices", 'exchange = np.einsum("ajP,biP->aibj", Bvo, Bvo)',
     'exchange = np.einsum("aiP,bjP->aibj", Bvo, Bvo)'),
    ("Z-vector orbital energy gap sign", "np.diag(((eps_vir[:, None] - eps_occ[None, :]) / 2.0)",
     "np.diag(((eps_occ[None, :] - eps_vir[:, None]) / 2.0)"),
    ("Z-vector L' transposed", "rhs = L2[:, :nocc] - L1[:, nocc:].T", "rhs = L2[:, :nocc] - L2[:, :nocc]"),
    ("W misses the HF density", "D[:nocc, :nocc] += np.eye(nocc)", "D[:nocc, :nocc] += 0.0"),
    ("W puts L'' on the occupied rows", "W[nocc:] += L2", "W[nocc:] += 0.0"),
    ("skip mask read one way only", "(skip[k][j] or skip[j][k])", "skip[k][j]"),
    ("skipped pair still computed", "continue            # screened out", "pass            # screened out"),
    ("pair_energy uses X", "V, X, T = pair_quantities(B, eps_occ, eps_vir, i, j)\n    return np.sum(T * V)",
     "V, X, T = pair_quantities(B, eps_occ, eps_vir, i, j)\n    return np.sum(T * X)"),
]


def load_mutant(old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found: %r" % old
    src = src.replace(old, new, 1)
    mod = types.ModuleType("rimp2_oracle_mutant")
    exec(compile(src, "<mutant>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    M = load_mutant(old, new)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(M)
        except Exception:
            caught.append(pin.__name__)
    assert caught, "planted mistake %r passes every pin" % name
