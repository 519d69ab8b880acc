"""The C ABI on the host: the library loads, exports every symbol the header
declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

import seeded_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(ntt_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2405_11353_amd as ntt
    return ntt.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def u64s(vals):
    return (ctypes.c_uint64 * len(vals))(*vals)


def test_plan_argument_validation(lib):
    q = si.ntt_primes(60, 18, 1)[0]
    lib.ntt_plan_create_ex.restype = ctypes.c_void_p
    lib.ntt_plan_create_ex.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
    cases = [
        ((1000, u64s([q]), 1, 0, None), -2),          # N not a power of two
        ((1 << 18, u64s([q]), 1, 0, None), -2),       # N too large
        ((1, u64s([q]), 1, 0, None), -2),
        ((1024, u64s([q + 2]), 1, 0, None), -3),      # not prime
        ((1024, u64s([q]), 1, 0x1, None), -3),        # too large for 32-bit words
        ((4096, u64s([12289]), 1, 0, None), -3),      # 2N does not divide q-1
        ((1024, u64s([(1 << 61) + 1]), 1, 0, None), -3),
        ((1024, None, 1, 0, None), -1),
        ((1024, u64s([q]), 0, 0, None), -1),
        ((1024, u64s([q]), 1, 0x80, None), -1),       # unknown flag
        ((1024, u64s([q]), 1, 0x10, None), -1),
        ((1024, u64s([q]), 1, 0, u64s([2])), -1),     # not a primitive 2N-th root
    ]
    for args, code in cases:
        assert lib.ntt_plan_create_ex(*args) is None
        assert lib.ntt_last_error() == code, (args, lib.ntt_last_error())


def test_plan_queries_reject_null_plans(lib):
    """The per-call variant queries check their plan and batch before reading
    anything (no GPU needed)."""
    out = ctypes.c_int32()
    p = ctypes.byref(out)
    assert lib.ntt_plan_get_col_tile(None, 1, p) == -1
    assert lib.ntt_plan_get_row_form(None, 1, p, p) == -1
    assert lib.ntt_plan_get_variant_for(None, 1, p, p, p) == -1


def test_strerror_covers_codes(lib):
    lib.ntt_strerror.restype = ctypes.c_char_p
    for c in range(0, -12, -1):
        assert lib.ntt_strerror(c) and lib.ntt_strerror(c) != b"unknown error"


def test_tune_table_save_load_round_trip(lib, tmp_path):
    import paper_2405_11353_amd as ntt
    ntt.ntt_tune_clear()
    f = tmp_path / "t.json"
    ntt.ntt_tune_save(str(f))          # empty table
    assert '"entries"' in f.read_text()
    with pytest.raises(ntt.NttError):
        ntt.ntt_tune_load(str(f))      # no entries
    arch = f.read_text().split('"arch": "')[1].split('"')[0]
    f.write_text('{"arch": "%s", "entries": [\n {"word": 64, "log_n": 16, "items_log2": 6, "path": 3, '
                 '"log_n1": 7, "exact": 0, "us": 12.5}]}' % arch)
    ntt.ntt_tune_load(str(f))
    ntt.ntt_tune_save(str(f))
    assert '"log_n1": 7' in f.read_text()
    f.write_text('{"arch": "gfx000", "entries": [{"word": 64, "log_n": 16, "items_log2": 6, "path": 3, '
                 '"log_n1": 7, "exact": 0, "us": 1}]}')
    with pytest.raises(ntt.NttError):
        ntt.ntt_tune_load(str(f))      # another architecture
    ntt.ntt_tune_clear()


def test_bconv_argument_validation(lib):
    ps = si.ntt_primes(60, 17, 70)
    lib.ntt_bconv_create.restype = ctypes.c_void_p
    lib.ntt_bconv_create.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                     ctypes.c_uint32]
    cases = [
        ((64, None, 1, u64s(ps[1:2]), 1), -1),
        ((64, u64s(ps[:1]), 0, u64s(ps[1:2]), 1), -1),        # empty source basis
        ((64, u64s(ps[:1]), 1, u64s(ps[1:2]), 0), -1),        # empty target basis
        ((64, u64s(ps[:65]), 65, u64s(ps[65:66]), 1), -1),    # source basis above 64 primes
        ((63, u64s(ps[:2]), 2, u64s(ps[2:3]), 1), -2),        # odd N
        ((0, u64s(ps[:2]), 2, u64s(ps[2:3]), 1), -2),
        ((64, u64s([ps[0], ps[0] + 2]), 2, u64s(ps[2:3]), 1), -3),   # not prime
        ((64, u64s(ps[:2]), 2, u64s([ps[1]]), 1), -3),        # repeated across the bases
        ((64, u64s([(1 << 61) + 1]), 1, u64s(ps[2:3]), 1), -3),
    ]
    for args, code in cases:
        assert lib.ntt_bconv_create(*args) is None
        assert lib.ntt_last_error() == code, (args, lib.ntt_last_error())


def _local_table(tmp_path):
    """The shipped gfx950 tuning table, relabelled with this machine's arch so the loader parses it."""
    import paper_2405_11353_amd as ntt
    f = tmp_path / "arch.json"
    ntt.ntt_tune_clear()
    ntt.ntt_tune_save(str(f))
    arch = f.read_text().split('"arch": "')[1].split('"')[0]
    src = open(os.path.join(ROOT, "paper_2405_11353_amd", "tune_gfx950.json")).read()
    return src.replace('"arch": "gfx950"', '"arch": "%s"' % arch)


def test_tune_load_rejects_out_of_range_fields(lib, tmp_path):
    import paper_2405_11353_amd as ntt
    good = _local_table(tmp_path)
    f = tmp_path / "t.json"
    f.write_text(good)
    ntt.ntt_tune_load(str(f))
    entry = '{"word": 64, "log_n": 16, "items_log2": 6, "path": 3, "log_n1": 8, "exact": 0, "us": 12.5}'
    head = good.split('"entries"')[0] + '"entries": ['
    bad = [("64", "48"), ('"log_n": 16', '"log_n": 40'), ('"log_n": 16', '"log_n": -1'),
           ('"items_log2": 6', '"items_log2": 1e300'), ('"path": 3', '"path": 9'),
           ('"log_n1": 8', '"log_n1": 12'), ('"exact": 0', '"exact": 2'), ('12.5', 'nan'),
           ('12.5', '-3'), ('"us": 12.5', '"us" 12.5'), ('"log_n": 16', '"log_n": x')]
    for old, new in bad:
        f.write_text(head + entry.replace(old, new, 1) + "]}")
        with pytest.raises(ntt.NttError):
            ntt.ntt_tune_load(str(f))
    for broken in ['{"arch": ', '{"arch"', '{"arch": "x', '']:
        f.write_text(broken)
        with pytest.raises(ntt.NttError):
            ntt.ntt_tune_load(str(f))
    ntt.ntt_tune_clear()


def test_tune_load_survives_damaged_tables(lib, tmp_path):
    """Truncated, byte-flipped and spliced copies of a valid table either load or
    raise; none may crash the loader."""
    import paper_2405_11353_amd as ntt
    good = _local_table(tmp_path).encode()
    f = tmp_path / "t.json"
    rng = si.Stream(2024)
    loaded = rejected = 0
    for it in range(400):
        v = bytearray(good)
        pos = [rng.uniform_int(0, len(v) - 1) for _ in range(8)]
        kind = it % 4
        if kind == 0:
            del v[pos[0]:]
        elif kind == 1:
            for p, b in zip(pos[:4], pos[4:]):
                v[p] = b & 0xFF
        elif kind == 2:
            for p, b in zip(pos[:4], pos[4:]):
                v[p] = b'{}[],:"0123456789-eE.x '[b % 23]
        else:
            a, b = sorted(pos[:2])
            del v[a:b]
        f.write_bytes(bytes(v))
        try:
            ntt.ntt_tune_load(str(f))
            loaded += 1
        except ntt.NttError:
            rejected += 1
        ntt.ntt_tune_clear()
    assert loaded + rejected == 400 and loaded > 0 and rejected > 0


def test_tune_table_row_form_and_values_per_thread_fields(lib, tmp_path):
    """Entries carry the tuned row form and the column passes' values per
    thread and columns per tile; they survive a save and load, tables without
    them still load, and values out of range drop the entry."""
    import paper_2405_11353_amd as ntt
    ntt.ntt_tune_clear()
    f = tmp_path / "t.json"
    ntt.ntt_tune_save(str(f))
    arch = f.read_text().split('"arch": "')[1].split('"')[0]
    head = '{"arch": "%s", "entries": [' % arch
    e = '{"word": 64, "log_n": 16, "items_log2": 6, "path": 3, "log_n1": 8, "exact": 0, "us": 9.5%s}'
    f.write_text(head + e % ', "row_twist": 3, "lv_col": 4, "col_tile": 32' + "]}")
    ntt.ntt_tune_load(str(f))
    ntt.ntt_tune_save(str(f))
    assert '"row_twist": 3, "lv_col": 4, "col_tile": 32' in f.read_text()
    f.write_text(head + e % ', "col_tile": 16' + "]}")   # 16 is the default tile
    ntt.ntt_tune_clear()
    ntt.ntt_tune_load(str(f))
    ntt.ntt_tune_save(str(f))
    assert '"col_tile": 0' in f.read_text()
    f.write_text(head + e % "" + "]}")                  # an older table: no new fields
    ntt.ntt_tune_clear()
    ntt.ntt_tune_load(str(f))
    ntt.ntt_tune_save(str(f))
    assert '"row_twist": -1, "lv_col": 0, "col_tile": 0' in f.read_text()
    for bad in (', "row_twist": 4', ', "row_twist": -2', ', "lv_col": 5', ', "lv_col": 2', ', "col_tile": 24',
                ', "col_tile": -16'):
        f.write_text(head + e % bad + "]}")
        ntt.ntt_tune_clear()
        with pytest.raises(ntt.NttError):
            ntt.ntt_tune_load(str(f))
    ntt.ntt_tune_clear()
