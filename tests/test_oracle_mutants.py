"""Each pin bites: a copy of the oracle with one planted mistake (see
tests/mutants.py) fails the pin that covers the function it alters, while the
oracle itself passes it (the pin's own test).  CPU only."""
from __future__ import annotations

import pytest

import mutants
import test_oracle_pins_emission as PE
import test_oracle_pins_fields as PF
import test_oracle_pins_ions as PI
import test_oracle_pins_pairs as PP

# mutant -> the pin that must catch it
CASES = [
    ("deposit2d_jx_weight", PF.check_continuity),
    ("deposit3d_T_weight", PF.check_continuity),
    ("deposit2d_jz_weights", PF.check_jz_path_average),
    ("current_quantum_2e-30", PF.check_continuity),
    ("gather_stagger_sign", PF.check_gather_multilinear),
    ("gather3d_z_fraction", PF.check_gather_multilinear),
    ("bhalf_curl_sign", PF.check_yee_modes),
    ("efull_curl_index", PF.check_yee_modes),
    ("mur_coefficient_sign", PF.check_mur_absorbs),
    ("source3d_amplitude", lambda lib: PF.check_gaussian_beam(3, lib)),
    ("source2d_gouy", lambda lib: PF.check_gaussian_beam(2, lib)),
    ("source_curvature_sign", lambda lib: PF.check_gaussian_beam(2, lib)),
    ("eta_pxB_sign", PE.check_eta_closed_forms),
    ("eta_pE_sign", PE.check_eta_closed_forms),
    ("eta_gamma_dropped", PE.check_eta_closed_forms),
    ("ncs_rate_blend", PE.check_ncs_rate_off_node),
    ("ncs_row_blend", PE.check_ncs_sampling_quantum),
    ("ncs_row_search", PE.check_ncs_sampling_quantum),
    ("brem_sigma_blend", PE.check_brem_sigma_off_node),
    ("brem_row_blend", PE.check_brem_sampling_off_node),
    ("brem_energy_map", PE.check_brem_sampling_off_node),
    ("exp_series_short", PE.check_math_against_libm),
    ("log_split_dropped", PE.check_math_against_libm),
    ("ion_push_charge_sign", PI.check_ion_gyration),
    ("ion_mass_dropped", PI.check_two_fluid_plasma_frequency),
    ("ion_deposit_charge", PI.check_continuity_with_ions),
    ("ion_density_volume", PI.check_brem_with_counted_ion_density),
    ("chi_cross_sign", PP.check_bw_conversion_law),
    ("bw_rate_alpha", PP.check_bw_conversion_law),
    ("bh_density_dropped", PP.check_bh_conversion_law),
    ("bw_share_row_length", PP.check_pair_shares),
    ("photon_move_sign", PP.check_pair_kinematics),
    ("spectrum_bin_offset", PE.check_spectrum_bins),
    ("K_BR_factor", PE.check_constants),
    ("E_S_factor", PE.check_constants),
]


@pytest.mark.parametrize("name,check", CASES, ids=[c[0] for c in CASES])
def test_planted_error_fails_its_pin(oracle_lib, name, check):
    lib = mutants.build(name)
    with pytest.raises(AssertionError):
        check(lib)


def test_every_mutant_has_a_pin():
    assert sorted(mutants.MUTANTS) == sorted(c[0] for c in CASES)
