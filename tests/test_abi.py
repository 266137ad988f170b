"""The C-ABI library loads and exports every entry point include/chem.h
declares (no GPU needed), and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "chem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chem_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    from paper_2112_05834_amd import chem
    L = chem.lib()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_mechanism_parse_and_errors(tmp_path):
    from paper_2112_05834_amd import chem, synth
    mech, path = synth.mech_cached("spray54", str(tmp_path))
    M = chem.Mechanism(path)
    assert (M.n_species, M.n_reactions) == (54, 269)
    w = M.work()
    assert w["flops_rhs"] > 1000 and w["flops_jac"] > w["flops_rhs"]
    bad = tmp_path / "bad.mech"
    bad.write_text(open(path).read().replace("reactions 269", "reactions 270"))
    with pytest.raises(chem.ChemError) as e:
        chem.Mechanism(str(bad))
    assert e.value.code == -2
    with pytest.raises(chem.ChemError):
        chem.Mechanism(str(tmp_path / "missing.mech"))


def test_opts_validation_without_device(tmp_path):
    from paper_2112_05834_amd import chem, synth
    _, path = synth.mech_cached("tiny9", str(tmp_path))
    M = chem.Mechanism(path)
    L = chem.lib()
    h = ctypes.c_void_p()
    for kw in [dict(rtol=0.0), dict(atol=-1.0), dict(max_steps=0), dict(schedule=7), dict(cells_per_wave=3)]:
        o = chem.default_opts(**kw)
        rc = L.chem_solver_create(M._h, ctypes.byref(o), 0, ctypes.byref(h))
        assert rc == -1, kw


def test_default_opts():
    from paper_2112_05834_amd import chem
    o = chem.default_opts()
    assert (o.rtol, o.atol, o.max_steps, o.schedule) == (1e-6, 1e-10, 100000, 0)


def test_null_and_bad_arguments_are_errors_not_crashes():
    from paper_2112_05834_amd import chem
    L = chem.lib()
    h = ctypes.c_void_p()
    assert L.chem_mech_load(None, ctypes.byref(h)) == -1
    assert L.chem_solver_create(None, None, 0, ctypes.byref(h)) == -1
    assert L.chem_integrate(None, 1, 1e-6, None, None, None, None, None, None, None) == -1
    assert L.chem_model_train(None, 1, None, None, None, None) == -1
    assert L.chem_bin_order(None, 1, None, None, None, None) == -1
    n = ctypes.c_int32()
    assert L.chem_kernel_times(None, None, 0, ctypes.byref(n)) == -1
    assert L.chem_autotune(None, 1, None, 1e-6, None) == -1
    assert L.chem_autotune_cached(None, b"/tmp/x.jsonl", 1, None, 1e-6, None, ctypes.byref(n)) == -1
    assert L.chem_zone_config(None, None, None, None, 0.0, 0.0) == -1
    assert L.chem_mixture_fraction(None, 1, None, None, None) == -1
    assert L.chem_zone_bands(None, 0.1) == -1
    assert L.chem_integrate_zonal(None, 1, 1e-6, None, None, None, None, None, None, None, None) == -1
    assert L.chem_mech_elements(None, ctypes.byref(n), None) == -1
    assert L.chem_last_error()          # a message is set
    L.chem_mech_free(None)               # NULL-safe
    L.chem_solver_free(None)


def test_element_counts_match_the_generator(tmp_path):
    from paper_2112_05834_amd import chem, synth
    mech, path = synth.mech_cached("spray54", str(tmp_path))
    assert (chem.Mechanism(path).elements() == mech.elem).all()


def test_too_many_species_is_a_mechanism_error(tmp_path):
    """Species beyond what the kernels address (255) are rejected at load,
    with a message, not later on the device."""
    from paper_2112_05834_amd import chem
    poly = "2.5 0 0 0 0 100 4"
    lines = ["chemmech 1", "elements 1", "E0 0.001", "species 300"]
    for k in range(300):
        lines += ["S%d 0.001 200 1000 6000 1" % k, poly, poly]
    lines += ["reactions 0", "end"]
    p = tmp_path / "big.mech"
    p.write_text("\n".join(lines) + "\n")
    with pytest.raises(chem.ChemError) as e:
        chem.Mechanism(str(p))
    assert e.value.code == -2
    assert "species" in str(e.value)


def test_eval_counters_rejects_bad_arguments_without_device():
    from paper_2112_05834_amd import chem
    L = chem.lib()
    assert L.chem_eval_counters(None, None, None, 0) == -1                  # no solver
    # (a solver is needed for the rest; its checks come before any device work)
