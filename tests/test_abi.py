"""CPU-side checks of the C-ABI library: it loads, exports every entry point the
header declares, and its host-side validation answers without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "goldbach.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gb_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def gb():
    import paper_2603_07850_amd as g
    return g


def test_header_declares_the_boundary_calls():
    names = _declared()
    for n in ("gb_base_primes", "gb_verify_range", "gb_verify_batch", "gb_last_error",
              "gb_is_prime_u64", "gb_autotune", "gb_release"):
        assert n in names


def test_library_exports_every_declared_symbol(gb):
    L = gb.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_header(gb):
    from paper_2603_07850_amd import _binding as b
    assert ctypes.sizeof(b.Result) == 11 * 8
    assert ctypes.sizeof(b.Params) == 24
    assert ctypes.sizeof(b.Stats) == 72


def test_no_table_is_reported_not_crashed(gb):
    gb.release()
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range(4, 100, 100)
    assert e.value.name == "GB_ENOTABLE"
    assert "gb_base_primes" in gb.lib().gb_last_error().decode()
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_batch([(4, 100)], 100)
    assert e.value.name == "GB_ENOTABLE"
    assert gb.table_limit() == 0 and gb.table_count() == 0


def test_host_validation_of_params(gb):
    saved = gb.get_params()
    for bad in (dict(seg_log2=17), dict(seg_log2=21), dict(wg_size=128), dict(wg_size=2048),
                dict(window=2), dict(window=65537), dict(wg_per_cu=65), dict(bucket_log2=16),
                dict(bucket_log2=33)):
        args = dict(seg_log2=18, wg_size=256, window=4096, wg_per_cu=0)
        args.update(bad)
        with pytest.raises(gb.GoldbachError) as e:
            gb.set_params(**args)
        assert e.value.name == "GB_EINVAL"
    gb.set_params(seg_log2=20, wg_size=1024, window=0, wg_per_cu=1, bucket_log2=24, bucket_mib=512)
    assert gb.get_params() == dict(seg_log2=20, wg_size=1024, window=0, wg_per_cu=1,
                                   bucket_log2=24, bucket_mib=512)
    gb.set_params(**saved)
    assert gb.get_params() == saved


def test_host_validation_of_wide_chunk(gb):
    assert gb.get_wide_chunk_log2() == 26
    for bad in (0, 11, 31, 64):
        with pytest.raises(gb.GoldbachError) as e:
            gb.set_wide_chunk_log2(bad)
        assert e.value.name == "GB_EINVAL"
        assert gb.get_wide_chunk_log2() == 26
    for ok in (12, 30, 26):
        gb.set_wide_chunk_log2(ok)
        assert gb.get_wide_chunk_log2() == ok


def test_base_primes_rejects_limit_above_2_32(gb):
    with pytest.raises(gb.GoldbachError) as e:
        gb.base_primes(1 << 32)
    assert e.value.name == "GB_EINVAL"


def test_product_path_has_no_oracle_or_fallback():
    """The package never imports, loads or links the oracle."""
    pkg = os.path.join(ROOT, "paper_2603_07850_amd")
    pat = re.compile(r"(import\s+oracle|from\s+oracle|liboracle|gb_oracle|\boracle\.[a-z_]+\()")
    for dirpath, _, files in os.walk(pkg):
        if "__pycache__" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not pat.search(src), f


def test_build_flags_keep_miscompiled_forms_out():
    """The kernels are built without packed fp32 ops and without v_bitop3 (the
    compiler's fused three-input bitwise ops gave wrong probe masks)."""
    from paper_2603_07850_amd import build
    flags = " ".join(build.FLAGS)
    assert "-target-feature -Xclang -packed-fp32-ops" in flags
    assert "-target-feature -Xclang -bitop3-insts" in flags


def test_failure_hook_validates_its_argument(gb):
    with pytest.raises(gb.GoldbachError) as e:
        gb.debug_fail_next(3)
    assert e.value.name == "GB_EINVAL"
    gb.debug_fail_next(1)
    gb.debug_fail_next(0)           # cleared again: nothing pending for later tests


def test_set_allocator_validation(gb):
    from paper_2603_07850_amd import _binding as b
    L = gb.lib()
    a = b.ALLOC_FN(lambda n, s, u: None)
    assert L.gb_set_allocator(a, b.FREE_FN(), None) == 1          # GB_EINVAL: one of the two
    assert L.gb_set_allocator(b.ALLOC_FN(), b.FREE_FN(), None) == 0


def test_noalloc_without_table_is_reported(gb):
    gb.release()
    with pytest.raises(gb.GoldbachError) as e:
        gb.verify_range_noalloc(4, 100, 100)
    assert e.value.name == "GB_ENOTABLE"

