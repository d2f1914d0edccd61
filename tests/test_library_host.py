"""Host-side checks of libftwa that need no GPU: the library loads, exports
every symbol include/ftwa.h declares, and its host lattice builder and Fock
starts agree bit-exactly with the oracle's independent implementation."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "ftwa.h")).read()
    return sorted(set(re.findall(r"\b(ftwa_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2212_04352_amd as ft
    lib = ft.load()
    declared = _declared_symbols()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    from paper_2212_04352_amd._binding import EXPORTS
    assert sorted(EXPORTS) == declared


@pytest.mark.parametrize("kind,a,b", [("torus", 2, 3), ("torus", 3, 9), ("torus", 2, 2),
                                      ("torus", 5, 7), ("armchair", 10, 20), ("armchair", 3, 4),
                                      ("armchair", 6, 9), ("hex", 1, 0), ("hex", 2, 0),
                                      ("hex", 3, 0), ("hex", 4, 0), ("hex", 5, 0), ("hex", 6, 0)])
def test_lattice_tables_match_oracle(orc, kind, a, b):
    import paper_2212_04352_amd as ft
    lat = ft.Lattice(kind, a, b)
    ref = orc.Lattice(kind, a, b)
    assert lat.N == ref.N and lat.n_bonds == ref.n_bonds
    assert np.array_equal(lat.nbr, ref.nbr)
    assert np.array_equal(lat.deg, ref.deg)
    assert np.array_equal(lat.sub, ref.sub)


def test_custom_lattice_and_errors(orc):
    import paper_2212_04352_amd as ft
    bonds = [(0, 1), (1, 2), (2, 3), (3, 0)]
    lat = ft.Lattice("custom", 0, bonds=bonds, sublattice=[0, 1, 0, 1], n_sites=4)
    ref = orc.Lattice.from_bonds(4, bonds, [0, 1, 0, 1])
    assert np.array_equal(lat.nbr, ref.nbr) and np.array_equal(lat.deg, ref.deg)
    with pytest.raises(ft.FtwaError):
        ft.Lattice("custom", 0, bonds=[(0, 1), (0, 1)], sublattice=[0, 1], n_sites=2)
    with pytest.raises(ft.FtwaError):
        ft.Lattice("custom", 0, bonds=[(0, 1), (0, 2), (0, 3), (0, 4)], sublattice=[0] * 5,
                   n_sites=5)
    with pytest.raises(ft.FtwaError):
        ft.Lattice("torus", 1, 3)
    with pytest.raises(ft.FtwaError):
        ft.Lattice("torus", 12, 12)  # 288 sites > 255


@pytest.mark.parametrize("kind,a,b", [("torus", 2, 3), ("torus", 3, 9), ("armchair", 10, 20),
                                      ("hex", 4, 0)])
def test_fock_starts_match_oracle(orc, kind, a, b):
    import paper_2212_04352_amd as ft
    lat = ft.Lattice(kind, a, b)
    ref = orc.Lattice(kind, a, b)
    assert np.array_equal(lat.fock_start("neel"), orc.fock_start(ref, "neel"))
    for seed, inst in [(0x2212043520000002, 0), (0x2212043520000004, 17), (1, 2**20)]:
        assert np.array_equal(lat.fock_start("random", seed, inst),
                              orc.fock_start(ref, "random", seed, inst))


def test_argument_errors_without_gpu():
    """Host validation rejects bad arguments before touching a device."""
    import paper_2212_04352_amd._binding as b
    lib = b.load()
    arr = (b.Instance * 1)()
    assert lib.ftwa_sample(arr, 0, 1, 0, None) == -1
    assert lib.ftwa_evolve(arr, 1, 0.01, 10, 1, 0, None, None, 0, None) == -1
    assert lib.ftwa_observables(0, 1, 1, None, None, None, None, None, None) == -1
    assert b.ftwa_last_error()
