"""C ABI surface checks that need no GPU: every symbol declared in
include/chem.h is exported, and host-side argument validation reports the
documented error codes."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "chem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(chem_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2510_23993_amd as chem
    L = chem.lib()
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(chem.chem.EXPORTS)


def test_bad_mechanism_files_rejected(tmp_path):
    import paper_2510_23993_amd as chem
    from synth.mechfile import Reaction, format_mechanism
    from tests import toymech
    with pytest.raises(chem.ChemError) as ei:
        chem.Mechanism(str(tmp_path / "missing.mech"))
    assert ei.value.rc == -4
    m = toymech.isomer_AB()
    m.reactions.append(Reaction({"A": 1}, {"N2": 1}, A=1.0, b=0.0, Ea=0.0))
    p = tmp_path / "bad.mech"
    p.write_text(format_mechanism(m))
    with pytest.raises(chem.ChemError, match="balanced") as ei:
        chem.Mechanism(str(p))
    assert ei.value.rc == -4
    # a valid file without compiled one-lane kernels is accepted (data-driven
    # kernels); without a GPU the load then stops at the first HIP call
    p.write_text(format_mechanism(toymech.isomer_AB()))
    try:
        chem.Mechanism(str(p))
    except chem.ChemError as ex:
        assert ex.rc == -2, str(ex)


def test_null_arguments():
    import paper_2510_23993_amd as chem
    L = chem.lib()
    assert L.chem_set_option(None, b"algorithm", 1.0) == -1
    assert L.chem_load_mechanism(None, None) == -1
    assert L.chem_integrate(None, 0, None, None, None, 0, None, None, None, 1.0, 1.0, 1.0, None) == -1
    assert L.chem_integrate_noalloc(None, 0, None, None, None, 0, None, None, None, 1.0, 1.0, 1.0) == -1
    assert L.chem_mlp_take(None, -1, None, None, None, None, None) == -1
    assert L.chem_mlp_take(None, 5, None, None, None, None, None) == -1
    assert L.chem_mlp_take(None, 0, None, None, None, None, None) == 0   # nothing to gather
    assert L.chem_synchronize(None) == -1
    assert b"NULL" in L.chem_last_error()


def test_structure_hash_matches_codegen():
    # the C++ parser's structure hash must select the kernels generated from the
    # same file: loading M9 either succeeds (GPU present) or fails only at the
    # first HIP call, never with "no kernels compiled"
    import paper_2510_23993_amd as chem
    from synth.fields import M9_PATH
    try:
        chem.Mechanism(M9_PATH)
    except chem.ChemError as ex:
        assert ex.rc == -2, str(ex)
