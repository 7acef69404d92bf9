"""Host-side checks of libmdmrg (no GPU): the library loads, exports every
entry point declared in include/mdmrg.h, and its host-only model builders
(Eq. (2)/(3) on the torus, momentum basis, mode rotation of Sec. II.B)
agree with the oracle's independent builders."""
import os
import re

import numpy as np
import pytest

import seeded_inputs as si
from oracle import integrals as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'mdmrg.h')


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r'\b(mdmrg_[a-z0-9_]+)\s*\(', src)))


@pytest.fixture(scope='module')
def lib():
    from paper_2311_14106_amd import mdmrg
    return mdmrg.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    from paper_2311_14106_amd import mdmrg
    assert set(names) == set(mdmrg.EXPORTS), 'binding and header disagree'


@pytest.mark.parametrize('model,basis,Lx,Ly,t,u', [
    (0, 0, 4, 4, 1.0, 1.0), (0, 1, 4, 4, 1.0, 2.0), (1, 0, 3, 3, 1.0, 4.0),
    (1, 1, 3, 3, 1.0, 4.0), (0, 1, 4, 3, 0.7, 1.3), (1, 1, 4, 2, 1.0, 8.0)])
def test_lattice_builders_match_oracle(lib, model, basis, Lx, Ly, t, u):
    from paper_2311_14106_amd import mdmrg
    T, V = mdmrg.build_lattice(model, basis, Lx, Ly, t, u)
    f = {(0, 0): I.spinless_real_space, (0, 1): I.spinless_momentum,
         (1, 0): I.hubbard_real_space, (1, 1): I.hubbard_momentum}[(model, basis)]
    To, Vo = f(Lx, Ly, t, u)
    assert np.abs(T - To).max() < 1e-14
    assert np.abs(V - Vo).max() < 1e-14


@pytest.mark.parametrize('spin', [False, True])
def test_mode_rotation_matches_oracle(lib, spin):
    from paper_2311_14106_amd import mdmrg
    model = 1 if spin else 0
    T, V = mdmrg.build_lattice(model, 1, 3, 2, 1.0, 3.0)
    R = si.random_orthogonal(6, 2)
    T2, V2 = mdmrg.rotate_modes(R, T, V, spin)
    To, Vo = I.rotate(T, V, R, spinful=spin)
    assert np.abs(T2 - To).max() < 1e-13
    assert np.abs(V2 - Vo).max() < 1e-13


def test_rotation_rejects_non_orthogonal(lib):
    from paper_2311_14106_amd import mdmrg
    T, V = mdmrg.build_lattice(0, 0, 2, 2, 1.0, 1.0)
    with pytest.raises(mdmrg.MdmrgError) as e:
        mdmrg.rotate_modes(np.eye(4) * 1.1, T, V, False)
    assert e.value.code == mdmrg.EINVAL


def test_create_rejects_a_device_that_does_not_exist(lib):
    # an ordinal past any machine's device count: the call fails cleanly,
    # leaves no handle and says why
    import ctypes
    from paper_2311_14106_amd import mdmrg
    h = ctypes.c_void_p(1)
    st = lib.mdmrg_create(ctypes.byref(h), 1 << 20, None)
    assert st == mdmrg.EDEVICE
    assert h.value is None
    assert lib.mdmrg_last_error(None).decode().startswith('HIP error')
    assert lib.mdmrg_create(None, 0, None) == mdmrg.EINVAL


def test_binding_fails_loudly_without_the_library(tmp_path):
    from paper_2311_14106_amd import mdmrg
    with pytest.raises(RuntimeError, match='not built'):
        mdmrg.load(str(tmp_path / 'libmdmrg.so'))


def test_product_path_does_not_use_the_oracle():
    # the package (binding, build, traffic tool, C/HIP sources) never reaches
    # into oracle/: no import, no path, no fallback
    pkg = os.path.join(ROOT, 'paper_2311_14106_amd')
    hits = []
    for d, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(('.py', '.cpp', '.hip', '.h')):
                src = open(os.path.join(d, f)).read()
                if re.search(r'\boracle\b', src):
                    hits.append(os.path.relpath(os.path.join(d, f), ROOT))
    assert not hits, hits
