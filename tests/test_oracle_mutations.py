"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a flipped sign, a wrong operand
order) in a private copy of the oracle source, builds it, and runs the pin
suite against that copy: the suite has to fail.  The real oracle is untouched.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dcem_oracle.cpp")
PY = os.path.join(ROOT, "oracle", "oracle.py")

MUTATIONS = {
    "gamma_te_sign": ("g_te = (cos_t - root) / (cos_t + root);",
                      "g_te = (root - cos_t) / (cos_t + root);"),
    "gamma_tm_operands": ("g_tm = (eps_c * cos_t - root) / (eps_c * cos_t + root);",
                          "g_tm = (cos_t - eps_c * root) / (cos_t + eps_c * root);"),
    "conductivity_sign": ("cplx eps_c(m.eps_r, -m.sigma", "cplx eps_c(m.eps_r, m.sigma"),
    "dropped_4pi": ("lam / (4.0 * kPi * length)", "lam / (kPi * length)"),
    "phase_sign": ("std::polar(mag, -k0 * length)", "std::polar(mag, k0 * length)"),
    "basis_order": ("V3 p_out = cross(sv, kr);", "V3 p_out = cross(kr, sv);"),
    "reflect_factor": ("d = d - (2.0 * dot(d, n)) * n;", "d = d - dot(d, n) * n;"),
    "image_factor": ("img[j - 1] - (2.0 * dot(img[j - 1] - f.p, f.n))", "img[j - 1] - (1.0 * dot(img[j - 1] - f.p, f.n))"),
    # transmissions (caught by the variant pins)
    "transmission_power_factor": ("-sc.mats[fc.material].pen_db / 20.0", "-sc.mats[fc.material].pen_db / 10.0",
                                  "test_oracle_variants.py"),
    "transmission_mirrors": ("img[j] = trans[j - 1] ? img[j - 1] :", "img[j] = false ? img[j - 1] :",
                             "test_oracle_variants.py"),
    "reflection_limit_with_branches": ("if (refl == A.max_refl) break;", "if (refl > A.max_refl) break;",
                                       "test_oracle_variants.py"),
    "opaque_face_transmits": ("if (!std::isfinite(sc.mats[sc.faces[bface].material].pen_db)) break;", "",
                              "test_oracle_variants.py"),
    "refine_accepts_opaque": ("if (trans[j] && !std::isfinite(sc.mats[sc.faces[fid[j]].material].pen_db)) return out;",
                              "", "test_oracle_variants.py"),
    "tie_break": ("if (t < tb) { tb = t;", "if (t <= tb) { tb = t;"),
    "capture_clamp": ("s = std::max(0.0, std::min(s, tb));", "s = std::max(0.0, s);"),
    "theta_hat_sign": ("V3{u.z * u.x / rho, u.z * u.y / rho, -rho}",
                       "V3{u.z * u.x / rho, u.z * u.y / rho, rho}"),
    "attenuation_sign": ("std::pow(10.0, -atten_db_per_km", "std::pow(10.0, atten_db_per_km"),
    "golden_angle": ("kPi * (3.0 - std::sqrt(5.0))", "kPi * (3.0 + std::sqrt(5.0))"),
    "no_in_face_check": ("if (!inside) return out;", "(void)inside;"),
    "no_occlusion": ("if (m >= 0 && inside_t) hit = true;", "(void)inside_t;"),
    "no_side_check": ("if (!(s > 0.0 && s < 1.0)) return out;", ""),
    "xform_order": ("r = r + (double)row[3];", "r = r - (double)row[3];"),
    "tie_flag_dropped": ("flags |= SEG_TIE;", "(void)0;"),
    # the power gradients (caught by the gradient pins)
    "dgamma_tm_sign": ("d_tm = 2.0 * cos_t * (r - eps_c / (2.0 * r))",
                       "d_tm = 2.0 * cos_t * (r + eps_c / (2.0 * r))", "test_oracle_gradients.py"),
    "dgamma_te_root": ("d_te = -cos_t / (r * ctr * ctr);", "d_te = -cos_t / (ctr * ctr);",
                       "test_oracle_gradients.py"),
    "derivative_not_propagated": (
        "dE[m] = cadd(cscale(gte * cdot(dE[m], sv), sv), cscale(gtm * cdot(dE[m], p_in), p_out));",
        "(void)m;", "test_oracle_gradients.py"),
    # the transmit pattern (caught by the pattern pins)
    "pattern_half_width": ("return std::max(0.0, 1.0 - d / step);",
                           "return std::max(0.0, 1.0 - 2.0 * d / step);", "test_oracle_pattern.py"),
    "pattern_azimuth_axes": ("const double phi = std::atan2(u.y, u.x);",
                             "const double phi = std::atan2(u.x, u.y);", "test_oracle_pattern.py"),
    "pattern_on_power": ("* pattern_gain(pattern, out.aod);",
                         "* pattern_gain(pattern, out.aod) * pattern_gain(pattern, out.aod);",
                         "test_oracle_pattern.py"),
}

# Mistakes planted in the Python half of the oracle (the per-receiver sums,
# the keys of records traced backward).
PY_MUTATIONS = {
    # incoherent power as the coherent one (square of the sum over paths)
    "p_inc_square_of_sum": ("return p_coh, p_inc", "return p_coh, p_coh.copy()"),
    # squared sum of component magnitudes instead of the sum of their squares
    "p_inc_component_sum": ("p_inc[:, t, r] += np.sum(np.abs(paths.amp[i]) ** 2, axis=-1)",
                            "p_inc[:, t, r] += np.sum(np.abs(paths.amp[i]), axis=-1) ** 2"),
    # coherent sum over only the last path of a receiver
    "p_coh_last_path": ("acc[:, int(paths.keys[i, 0]), int(paths.keys[i, 1])] += paths.amp[i]",
                        "acc[:, int(paths.keys[i, 0]), int(paths.keys[i, 1])] = paths.amp[i]"),
    # backward records keyed without reversing their faces / swapping the pair
    "backward_faces_not_reversed": ("out[sel, 3:3 + o] = rows[sel, 3:3 + o][:, ::-1]",
                                    "out[sel, 3:3 + o] = rows[sel, 3:3 + o]", "test_oracle_variants.py"),
    "backward_pair_not_swapped": ("out[:, 0], out[:, 1] = rows[:, 1], rows[:, 0]",
                                  "out[:, 0], out[:, 1] = rows[:, 0], rows[:, 1]", "test_oracle_variants.py"),
    # visited series that skip a ray's first hit, or keep the receiver's face order
    "visited_series_offset": ("faces = tr.face[src_i, row_i, :d]", "faces = tr.face[src_i, row_i, 1:d + 1]",
                              "test_oracle_variants.py"),
    # visited series of a branch that repeat its parent's, or skip its transmission flags
    "visited_branch_flags": ("faces = np.where(tbits == 1, -2 - faces, faces)", "faces = faces + 0 * tbits",
                             "test_oracle_variants.py"),
    "visited_backward_not_reversed": ("faces = faces[:, ::-1]", "faces = faces[:, ::1]", "test_oracle_variants.py"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name][:2]
    suite = MUTATIONS[name][2] if len(MUTATIONS[name]) > 2 else "test_oracle_pins.py"
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: %s" % name
    mutated = src.replace(old, new)
    cpp = tmp_path / "mut.cpp"
    lib = tmp_path / "libmut.so"
    cpp.write_text(mutated)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread",
                           str(cpp), "-o", str(lib)])
    env = dict(os.environ, DCEM_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", suite)],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, "pins did not catch mutation %s:\n%s" % (name, r.stdout[-2000:])


def _run_pins_on_python_copy(tmp_path, old, new, suite="test_oracle_pins.py"):
    src = open(PY).read()
    assert src.count(old) == 1, "mutation anchor not found: %r" % old
    mod = tmp_path / "oracle_mutant.py"
    mod.write_text(src.replace(old, new).replace(
        '_HERE = os.path.dirname(os.path.abspath(__file__))',
        '_HERE = %r' % os.path.join(ROOT, "oracle")))
    env = dict(os.environ, DCEM_ORACLE_PY=str(mod))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", suite)],
                          env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)


def test_unmutated_python_copy_passes_the_pins(tmp_path):
    # control: the copy mechanism alone must not make the pins fail
    r = _run_pins_on_python_copy(tmp_path, "return p_coh, p_inc", "return p_coh, p_inc")
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(PY_MUTATIONS))
def test_pins_catch_python_mutation(name, tmp_path):
    r = _run_pins_on_python_copy(tmp_path, *PY_MUTATIONS[name])
    assert r.returncode == 1, "pins did not catch mutation %s:\n%s" % (name, r.stdout[-2000:])
    assert " failed" in r.stdout and " error" not in r.stdout, r.stdout[-2000:]
