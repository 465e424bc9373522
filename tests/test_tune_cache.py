"""Host-side tune-cache lookup (no GPU): the JSON-lines format written by
bfx_xengine_autotune, keyed by (device architecture, dtype, shape), the last
matching line winning."""
import paper_1708_00720_amd as bfx


def _write(tmp_path, lines):
    p = tmp_path / "tune.jsonl"
    p.write_text("".join(l + "\n" for l in lines))
    return str(p)


def test_lookup_matches_all_three_keys(tmp_path):
    path = _write(tmp_path, [
        '{"arch": "gfx950", "dtype": "ci4", "shape": "704x192", "variant": 1, "us": [240.0, 233.0]}',
        '{"arch": "gfx950", "dtype": "ci8", "shape": "704x192", "variant": 0, "us": [100.0, 110.0]}',
        '{"arch": "gfx942", "dtype": "ci4", "shape": "704x192", "variant": 0, "us": [1.0, 2.0]}',
    ])
    assert bfx.bfx_tune_cache_lookup(path, "gfx950", "ci4", "704x192") == 1
    assert bfx.bfx_tune_cache_lookup(path, "gfx950", "ci8", "704x192") == 0
    assert bfx.bfx_tune_cache_lookup(path, "gfx942", "ci4", "704x192") == 0
    assert bfx.bfx_tune_cache_lookup(path, "gfx950", "ci4", "704x191") == -1
    assert bfx.bfx_tune_cache_lookup(path, "gfx950", "cf16", "704x192") == -1


def test_last_matching_line_wins_and_bad_lines_are_skipped(tmp_path):
    path = _write(tmp_path, [
        '{"arch": "gfx950", "dtype": "ci8", "shape": "b:32x1024,64x512", "variant": 1, "us": [5.0, 4.0]}',
        'not json at all',
        '{"arch": "gfx950", "dtype": "ci8", "shape": "b:32x1024,64x512", "variant": 7, "us": []}',
        '{"arch": "gfx950", "dtype": "ci8", "shape": "b:32x1024,64x512", "variant": 0, "us": [4.0, 5.0]}',
        '{"arch": "gfx950", "dtype": "ci8", "shape": "b:32x1024", "variant": 1, "us": [9.0, 8.0]}',
    ])
    # variant 7 is out of range and ignored; the last valid match is 0
    assert bfx.bfx_tune_cache_lookup(path, "gfx950", "ci8", "b:32x1024,64x512") == 0
    assert bfx.bfx_tune_cache_lookup(path, "gfx950", "ci8", "b:32x1024") == 1


def test_missing_file_and_null_arguments(tmp_path):
    assert bfx.bfx_tune_cache_lookup(str(tmp_path / "absent.jsonl"), "gfx950", "ci4", "64x1") == -1
    assert bfx._lib.bfx_tune_cache_lookup(None, b"gfx950", b"ci4", b"64x1") == -1


def test_set_variant_range_checks():
    plan = bfx.bfx_xengine_create(64, 4, "ci8")
    try:
        nv = bfx.bfx_xengine_num_variants(plan)
        assert nv == 2  # ci8: int8 MFMA with four or eight DMA waves
        assert bfx.bfx_xengine_variant(plan) in range(nv)
        for v in range(nv):
            bfx.bfx_xengine_set_variant(plan, v)
            assert bfx.bfx_xengine_variant(plan) == v
        for bad in (-1, nv, bfx.BFX_XENGINE_VARIANTS):
            try:
                bfx.bfx_xengine_set_variant(plan, bad)
            except bfx.BfxError as e:
                assert e.status == bfx.BFX_EINVAL
            else:
                raise AssertionError("out-of-range variant accepted")
    finally:
        plan.close()
    assert bfx._lib.bfx_xengine_variant(None) == -1
    assert bfx._lib.bfx_xengine_num_variants(None) == -1
    p4 = bfx.bfx_xengine_create(64, 4, "ci4")
    try:
        assert bfx.bfx_xengine_num_variants(p4) == 4  # ci4 also has the FP8 variants
        bfx.bfx_xengine_set_variant(p4, 3)
        assert bfx.bfx_xengine_variant(p4) == 3
    finally:
        p4.close()


def test_autotune_rejects_bad_ntime():
    plan = bfx.bfx_xengine_create(64, 4, "ci8")
    try:
        for bad in (0, -5, bfx.bfx_xengine_max_ntime("ci8") + 1):
            try:
                bfx.bfx_xengine_autotune(plan, bad, stream=0)
            except bfx.BfxError as e:
                assert e.status == bfx.BFX_EINVAL
            else:
                raise AssertionError(f"ntime={bad} accepted")
    finally:
        plan.close()
