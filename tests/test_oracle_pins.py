"""The CPU oracle against facts fixed by the paper and by the mathematics.

Pin status of every oracle function:
  pair_integrals, denominators, amplitudes, combination, pair_quantities,
  fragment (all outputs)      brute force, closed form, equal energies,
                              dE/dB = 4 Gamma, dE/d eps = 2 diag P, invariants
  fragment(skip=...)          deleting an orbital, empty mask
  pair_energy, gamma_row, gamma_rows, p_ab_element, p_ij_element
                              brute force
  exact_sum                   exact cancellation cases
  gamma_metric                chain rule: dE/dB3 = 4 gamma_metric (complex step)
  gamma_ao                    chain rule through the MO transform (complex step)
  l_prime, l_dprime           orbital-mixing derivatives of E (complex step)
  antisym_term, zvector       brute force over the Appendix's index forms
                              (Gauss-Jordan solve), single-pair closed form
  energy_weighted_density     HF limit (eps_i on the occupied diagonal) and
                              brute force over the pieces as read
No function is unpinned.
"""
import pytest

from oracle import rimp2_oracle as O
import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(O)
