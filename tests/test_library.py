"""CPU checks of the C-ABI boundary: the library loads, exports every declared symbol,
and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rom.h")
LIB = os.path.join(ROOT, "paper_1602_00138_amd", "librom.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"ROM_API\s+[\w\s\*]+?\b(rom_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def R():
    if not os.path.exists(LIB):
        pytest.fail("librom.so not built (run __graft_entry__.build())")
    from paper_1602_00138_amd import rom
    return rom


def test_library_exports_every_declared_symbol(R):
    lib = ctypes.CDLL(LIB)
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(R.EXPORTED) == syms


def test_header_struct_sizes_match_binding(R):
    # rom_record / rom_stats are read field by field through ctypes
    assert ctypes.sizeof(R.rom_record) == 72
    assert ctypes.sizeof(R.rom_grid) == 48


@pytest.mark.parametrize("dim,N,bc,A", [(4, (3, 3, 3), (0,) * 6, 1.0), (2, (3, 3, 2), (0,) * 6, 1.0),
                                        (3, (0, 3, 3), (0,) * 6, 1.0), (3, (3, 3, 3), (0, 2, 0, 0, 0, 0), 1.0),
                                        (3, (3, 3, 3), (0,) * 6, -1.0)])
def test_invalid_grid_rejected(R, dim, N, bc, A):
    g = R.make_grid(dim, N, bc, A)
    with pytest.raises(R.RomError) as e:
        R.rom_operator_bytes(g, False)
    assert e.value.status == R.ROM_EINVAL


def test_operator_bytes(R):
    g = R.make_grid(3, (64, 64, 64), (0, 0, 0, 0, 1, 1), 1.0)
    n = 64 ** 3
    assert R.rom_operator_bytes(g, False) >= 8 * n
    assert R.rom_operator_bytes(g, True) >= 8 * 5 * n


def test_null_handles_rejected(R):
    opts = R.make_opts(1e-8)
    with pytest.raises(R.RomError) as e:
        R.rom_sequence_bytes(None, 4, 4, 10, 2, opts)
    assert e.value.status == R.ROM_EINVAL
    with pytest.raises(R.RomError):
        R.rom_basis_dims(None)


@pytest.mark.parametrize("g", [(12, 16, 16), (16, 16, 0), (16, 8, 4)])
def test_seednet_rejects_grids_not_multiple_of_8(R, g):
    with pytest.raises(R.RomError) as e:
        R.rom_seednet_bytes(*g, 1)
    assert e.value.status == R.ROM_EINVAL


def test_seednet_sizes(R):
    from paper_1602_00138_amd import seed
    npar, pb, wb = R.rom_seednet_bytes(16, 16, 16, 2)
    assert npar == seed.flatten(seed.unflatten(seed.he_init(0))).size
    assert pb >= 4 * 4 * npar and wb > 0


def test_seednet_outputs_and_subspace_sizes(R):
    from paper_1602_00138_amd import seed
    npar16, _, _ = R.rom_seednet_bytes(16, 16, 16, 2, 16)
    assert npar16 == seed.he_init(0, outputs=16).size
    npar1, _, _ = R.rom_seednet_bytes(16, 16, 16, 2, 1)
    assert npar16 - npar1 == 15 * (16 * 27 + 1)
    for bad in (0, 17):
        with pytest.raises(R.RomError):
            R.rom_seednet_bytes(16, 16, 16, 2, bad)
    assert R.rom_subspace_loss_bytes(1000, 16, 64) > 8 * 1000 * (16 + 64)
    for k, s in ((0, 4), (17, 4), (4, 0)):
        with pytest.raises(R.RomError):
            R.rom_subspace_loss_bytes(1000, k, s)

