"""The synthetic workloads sit in the two regimes the paper separates by depth of field
(Section 1: DOF = Delta^2/(2 lambda); Delta = 1/|q_max|, Section 2 before eq. 13): the diffraction
workloads have DOF below the object's thickness, so the Ewald-sphere curvature of
eqs. 8-11 matters, as in Section 3's first example; the CT workload has DOF far above it,
the limit where eq. 11 reduces to eqs. 13-15, as in Section 3's second example.  The
paper's own example values are in tests/golden/paper_regimes.json.  CPU only."""
import json
import math
import os

import pytest

from synth import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_regimes.json")))

# CODATA constants for the textbook relativistic electron wavelength
H = 6.62607015e-34
M_E = 9.1093837015e-31
C = 299792458.0
E_CH = 1.602176634e-19


def dof(delta, lam):
    return delta * delta / (2.0 * lam)


def electron_wavelength(energy_ev):
    e = energy_ev * E_CH
    return H / math.sqrt(2.0 * M_E * e * (1.0 + e / (2.0 * M_E * C * C)))


def test_first_example_is_consistent_with_the_dof_definition():
    """200 keV electrons: lambda ~ 0.025 A; a 40 mrad aperture passes q up to alpha/lambda,
    so Delta = lambda/alpha and DOF ~ 8 A, below the ~70 A particle (Section 3)."""
    ex = GOLD["diffraction_example"]
    lam_a = electron_wavelength(ex["energy_eV"]) * 1e10
    assert abs(lam_a - ex["wavelength_A"]) < 0.01 * ex["wavelength_A"]
    delta = lam_a / ex["objective_aperture_rad"]
    assert abs(dof(delta, lam_a) - ex["dof_A"]) < 0.05 * ex["dof_A"]
    assert ex["dof_A"] < ex["object_size_A"]
    assert GOLD["ct_example"]["dof_m"] > 100 * GOLD["ct_example"]["thickness_m"]


def _workload_dof_ratio(w):
    """DOF over the volume's edge, Delta = 1/q_max with q_max = 1/(2 pixel) (axis Nyquist)."""
    delta = 2.0 * w.voxel
    return dof(delta, w.wavelength) / (w.n_vox * w.voxel)


@pytest.mark.parametrize("name", ["dt_ewald_128", "xray_jitter_256"])
def test_diffraction_workloads_have_dof_below_thickness(name):
    w = workloads.WORKLOADS[name]
    assert w.ewald == 1 and w.image_model == "born"
    assert _workload_dof_ratio(w) < 1.0


def test_ct_workload_has_dof_far_above_thickness():
    w = workloads.WORKLOADS["ct_pct_64"]
    assert _workload_dof_ratio(w) > 100.0
    assert w.span_deg == GOLD["ct_example"]["span_deg"]
