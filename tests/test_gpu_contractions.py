"""chem_eval_contractions: the stoichiometric contractions of the matrix-form
rate evaluation (nu'^T ln C and nu''^T ln C per reaction) in FP64 and FP32
sparse form and on the BF16 matrix cores (three-term split of ln C), against
the same products formed in numpy from stoichiometric matrices read directly
from the mechanism file, on both mechanisms, with ragged batch sizes."""
import numpy as np
import pytest

from synth import fields
from tests.gpu_util import host, to_dev

pytestmark = pytest.mark.gpu


def stoich_from_file(path):
    """(species, nu' [ns][nr], nu'' [ns][nr]) from the REACTANTS / PRODUCTS
    records of a mechanism file."""
    tok = []
    for line in open(path):
        tok += line.split("#", 1)[0].split()
    i = tok.index("SPECIES")
    ns = int(tok[i + 1])
    i += 2
    species = []
    ne = int(tok[tok.index("ELEMENTS") + 1])
    for _ in range(ns):
        species.append(tok[i])
        i += 2 + ne
    idx = {s: k for k, s in enumerate(species)}
    cols_f, cols_r = [], []
    for j, t in enumerate(tok):
        if t == "REACTANTS":
            m = int(tok[j + 1])
            f = np.zeros(ns)
            for q in range(m):
                f[idx[tok[j + 2 + 2 * q]]] += float(tok[j + 3 + 2 * q])
            p = j + 2 + 2 * m
            assert tok[p] == "PRODUCTS"
            m2 = int(tok[p + 1])
            r = np.zeros(ns)
            for q in range(m2):
                r[idx[tok[p + 2 + 2 * q]]] += float(tok[p + 3 + 2 * q])
            cols_f.append(f)
            cols_r.append(r)
    return species, np.array(cols_f).T, np.array(cols_r).T


@pytest.mark.parametrize("path", [fields.M9_PATH, fields.M53_PATH])
@pytest.mark.parametrize("n", [1, 17, 4099])
def test_contractions_against_stoichiometric_matrices(path, n):
    import torch
    import paper_2510_23993_amd as chem
    species, nuf, nur = stoich_from_file(path)
    mech = chem.Mechanism(path)
    assert mech.species == species and nuf.shape == (mech.ns, mech.nr)
    ctx = chem.Context(mech)
    rng = np.random.default_rng(n + mech.ns)
    lnC = rng.uniform(-45.0, 8.0, (mech.ns, n))
    ref_f, ref_r = nuf.T @ lnC, nur.T @ lnC
    d_lnC = to_dev(lnC)
    scale = np.abs(nuf).T @ np.abs(lnC) + np.abs(nur).T @ np.abs(lnC)   # size of the sums
    for prec, tol in ((0, 1e-14), (1, 5e-7), (2, 5e-7)):
        zf = torch.full((mech.nr, n), float("nan"), dtype=torch.float64, device="cuda")
        zr = torch.full_like(zf, float("nan"))
        ctx.eval_contractions(d_lnC, zf, zr, prec)
        torch.cuda.synchronize()
        ef = np.abs(host(zf) - ref_f) / np.maximum(scale, 1.0)
        er = np.abs(host(zr) - ref_r) / np.maximum(scale, 1.0)
        print(f"{mech.ns} species, n {n}, precision {prec}: max relative error {max(ef.max(), er.max()):.2e}")
        assert np.all(np.isfinite(host(zf))) and np.all(np.isfinite(host(zr)))
        assert ef.max() <= tol and er.max() <= tol, (prec, ef.max(), er.max())


def test_contraction_arguments():
    import paper_2510_23993_amd as chem
    mech = chem.Mechanism(fields.M9_PATH)
    ctx = chem.Context(mech)
    L = chem.lib()
    assert L.chem_eval_contractions(ctx._h, 10, None, None, None, 0) == -1
    assert L.chem_eval_contractions(ctx._h, 10, None, None, None, 3) == -1
    assert L.chem_eval_contractions(ctx._h, 0, None, None, None, 2) == 0
