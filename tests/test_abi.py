"""C-ABI checks that need no GPU: the library loads, exports every function declared in
include/gbb.h, and rejects invalid arguments on the host before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

L = pytest.importorskip("paper_2412_12734_amd._lib")


def _lib():
    try:
        return L.load()
    except ImportError as e:  # not built in this checkout
        pytest.skip(str(e))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gbb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gb_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert set(declared_functions()) == set(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_sizes_match_header_layout():
    # gb_view: 2 ints + 4 floats + 9 + 3 + 1 floats
    assert ctypes.sizeof(L.GbView) == 4 * (2 + 4 + 9 + 3 + 1)
    assert ctypes.sizeof(L.GbOptions) == 4 * (5 + 3 + 6)
    # P, N, tex_dtype, pad, six pointers, sh_degree, pad, sh, tex_side, tex_offset, n_texels
    assert ctypes.sizeof(L.GbSplats) == 16 + 6 * 8 + 8 + 8 + 3 * 8
    assert L.GbSplats.sh.offset == 16 + 6 * 8 + 8
    assert L.GbSplats.n_texels.offset == 16 + 6 * 8 + 8 + 8 + 2 * 8
    assert ctypes.sizeof(L.GbGrads) == 7 * 8
    assert ctypes.sizeof(L.GbLayout) == 8 * 20


def test_default_options():
    lib = _lib()
    o = L.GbOptions()
    lib.gb_default_options(ctypes.byref(o))
    assert o.sigma == pytest.approx(0.5)
    assert o.alpha_min == np.float32(1 / 255)
    assert o.alpha_max == pytest.approx(0.99)
    assert o.t_min == pytest.approx(1e-4)
    assert (o.tile_w, o.tile_h, o.batch, o.batch_bwd, o.prefix_pairs_per_tile,
            o.tile_order) == (16, 16, 0, 0, 0, 0)


def _layout(P=100, N=4, views=None, opts=None, cap=1000):
    lib = _lib()
    views = views or [sg.look_at_view((0, 0, -3), 64, 48)]
    lay = L.GbLayout()
    st = lib.gb_workspace_layout(P, N, L.make_views(views), len(views),
                                 ctypes.byref(opts or L.make_options()), cap, ctypes.byref(lay))
    return st, lay


def test_layout_sections_are_aligned_and_disjoint():
    views = [sg.look_at_view((0, 0, -3), 64, 48), sg.look_at_view((1, 0, -3), 33, 17)]
    st, lay = _layout(P=1000, views=views, cap=12345)
    assert st == L.GB_OK
    offs = [lay.status, lay.depth_key, lay.tile_count, lay.records, lay.order, lay.pair_keys,
            lay.pair_vals, lay.ranges, lay.n_last, lay.pair_keys_rest, lay.pair_vals_rest,
            lay.ranges_rest, lay.n_last_rest, lay.open_tiles, lay.tile_order, lay.tile_work]
    assert all(o % 256 == 0 for o in offs)
    assert len(set(offs)) == len(offs)
    assert max(offs) < lay.total_bytes
    assert lay.pair_capacity == 12345
    assert lay.total_tiles == 4 * 3 + 3 * 2
    # the depth-prefix pass gets 1024 pairs per tile by default, rounded up to 1024 slots
    assert lay.prefix_capacity == 18 * 1024
    assert lay.pair_keys_rest == lay.pair_keys + 4 * lay.prefix_capacity


def test_tile_order_sections_follow_the_option():
    views = [sg.look_at_view((0, 0, -3), 64, 48)]
    st, lay = _layout(P=1000, views=views, cap=5000)
    assert st == L.GB_OK
    # default: work-ordered backward, with its order and the forward's spans in the workspace
    assert lay.tile_order % 256 == 0 and lay.tile_work % 256 == 0
    assert 0 < lay.tile_order < lay.tile_work < lay.total_bytes
    o = L.make_options(tile_order=-1)
    st, lay2 = _layout(P=1000, views=views, opts=o, cap=5000)
    assert st == L.GB_OK and lay2.tile_order == 0 and lay2.tile_work == 0
    assert lay2.total_bytes <= lay.total_bytes


@pytest.mark.parametrize("field,value,status", [
    ("tile_w", 12, L.GB_ERR_ARG), ("tile_h", 64, L.GB_ERR_ARG), ("batch", 7, L.GB_ERR_ARG),
    ("batch_bwd", 64, L.GB_ERR_ARG), ("prefix_pairs_per_tile", -2, L.GB_ERR_ARG),
    ("tile_order", 2, L.GB_ERR_ARG), ("tile_order", -2, L.GB_ERR_ARG),
    ("sigma", 0.0, L.GB_ERR_ARG), ("alpha_max", 1.5, L.GB_ERR_ARG), ("t_min", -1.0, L.GB_ERR_ARG),
    ("lowpass_var", 0.0, L.GB_ERR_ARG),
])
def test_invalid_options_are_rejected(field, value, status):
    o = L.make_options()
    setattr(o, field, value)
    st, _ = _layout(opts=o)
    assert st == status


def test_invalid_sizes_are_rejected():
    assert _layout(P=0)[0] == L.GB_ERR_ARG
    assert _layout(N=3)[0] == L.GB_ERR_UNSUPPORTED
    assert _layout(N=32)[0] == L.GB_ERR_UNSUPPORTED
    # N = 16 is built with batches of 4 only, and batches of 4 for N = 16 only
    assert _layout(N=16)[0] == L.GB_OK
    assert _layout(N=16, opts=L.make_options(batch=4, batch_bwd=4))[0] == L.GB_OK
    assert _layout(N=16, opts=L.make_options(batch=8))[0] == L.GB_ERR_UNSUPPORTED
    assert _layout(N=16, opts=L.make_options(batch_bwd=8))[0] == L.GB_ERR_UNSUPPORTED
    assert _layout(N=16, opts=L.make_options(batch=16))[0] == L.GB_ERR_UNSUPPORTED
    assert _layout(N=8, opts=L.make_options(batch=4))[0] == L.GB_ERR_UNSUPPORTED
    assert _layout(N=8, opts=L.make_options(batch_bwd=4))[0] == L.GB_ERR_UNSUPPORTED
    assert _layout(N=8, opts=L.make_options(batch=2))[0] == L.GB_ERR_ARG
    assert _layout(cap=-1)[0] == L.GB_ERR_ARG
    bad = sg.look_at_view((0, 0, -3), 0, 48)
    assert _layout(views=[bad])[0] == L.GB_ERR_ARG


def test_render_rejects_null_pointers_before_launching():
    lib = _lib()
    views = L.make_views([sg.look_at_view((0, 0, -3), 32, 32)])
    sp = L.GbSplats(10, 4, L.GB_F32, None, None, None, None, None, None)
    opts = L.make_options()
    st = lib.gb_render_fwd(ctypes.byref(sp), views, 1, ctypes.byref(opts), None, 0, 0, None,
                           None, None)
    assert st == L.GB_ERR_ARG
    assert b"NULL" in lib.gb_last_error()


def test_mixed_grid_sides_are_checked_before_launching():
    """Grids of several sides need the layout side 8 or 16, a tex_offset array and n_texels;
    each refusal comes before any device access."""
    lib = _lib()
    views = L.make_views([sg.look_at_view((0, 0, -3), 32, 32)])
    opts = L.make_options()
    buf = ctypes.create_string_buffer(256)
    base = ctypes.addressof(buf)
    p16 = base + (-base) % 16

    def fwd(N, side, offset, n_texels):
        sp = L.GbSplats(10, N, L.GB_F32, p16, p16, p16, p16, p16, p16, 0, None, side, offset,
                        n_texels)
        return lib.gb_render_fwd(ctypes.byref(sp), views, 1, ctypes.byref(opts), None, 0, 0,
                                 None, None, None)

    assert fwd(4, p16, p16, 100) == L.GB_ERR_UNSUPPORTED  # layout side must be 8 or 16
    assert b"8 or 16" in lib.gb_last_error()
    assert fwd(8, p16, None, 100) == L.GB_ERR_ARG  # offsets missing
    assert fwd(16, p16, p16, 0) == L.GB_ERR_ARG  # no texels
    assert fwd(8, p16 + 2, p16, 100) == L.GB_ERR_ARG  # misaligned sides
    # the sides' checks passed: the next refusal is the missing workspace
    assert fwd(8, p16, p16, 100) == L.GB_ERR_ARG and b"workspace" in lib.gb_last_error()


def test_training_glue_rejects_invalid_arguments_before_any_launch():
    lib = _lib()
    assert lib.gb_activate_fwd(-1, *([None] * 7), None) == L.GB_ERR_ARG
    assert lib.gb_activate_fwd(0, *([None] * 7), None) == L.GB_OK  # nothing to do
    assert lib.gb_activate_bwd(5, *([None] * 10), None) == L.GB_ERR_ARG
    assert lib.gb_l1_loss(10, None, None, 1.0, None, None, None) == L.GB_ERR_ARG
    buf = ctypes.create_string_buffer(64)
    base = ctypes.addressof(buf)
    p16 = base + (-base) % 16
    # misaligned (4 bytes past a 16-byte boundary) arrays are refused
    assert lib.gb_l1_loss(4, p16 + 4, p16, 1.0, p16, p16, None) == L.GB_ERR_ARG
    assert lib.gb_adam_step(4, p16, p16, p16, p16, 0, 0.1, 0.9, 0.999, 1e-15, None,
                            None) == L.GB_ERR_ARG  # step must be >= 1
    assert lib.gb_adam_step(4, p16, p16, p16, p16, 1, 0.1, 1.0, 0.999, 1e-15, None,
                            None) == L.GB_ERR_ARG  # beta1 must be < 1
    assert lib.gb_adam_step(0, None, None, None, None, 1, 0.1, 0.9, 0.999, 1e-15, None,
                            None) == L.GB_OK  # empty
    assert lib.gb_to_bf16(-1, None, None, None) == L.GB_ERR_ARG



def test_image_fitting_glue_rejects_invalid_arguments_before_any_launch():
    lib = _lib()
    buf = ctypes.create_string_buffer(64)
    base = ctypes.addressof(buf)
    p16 = base + (-base) % 16
    assert lib.gb_mse_loss(-1, p16, p16, 1.0, p16, p16, None) == L.GB_ERR_ARG
    assert lib.gb_mse_loss(4, p16 + 4, p16, 1.0, p16, p16, None) == L.GB_ERR_ARG  # misaligned
    assert lib.gb_mse_loss(4, None, p16, 1.0, p16, p16, None) == L.GB_ERR_ARG
    for N, M in ((8, 3), (4, 8), (128, 2), (0, 1), (8, 0)):
        assert lib.gb_box_filter_textures(2, N, M, p16, p16, None) == L.GB_ERR_ARG, (N, M)
    assert lib.gb_box_filter_textures(-1, 8, 2, p16, p16, None) == L.GB_ERR_ARG
    assert lib.gb_box_filter_textures(2, 8, 2, None, p16, None) == L.GB_ERR_ARG
    assert lib.gb_box_filter_textures(0, 8, 2, None, None, None) == L.GB_OK  # nothing to do
    assert lib.gb_rotz_only(-1, p16, None) == L.GB_ERR_ARG
    assert lib.gb_rotz_only(3, None, None) == L.GB_ERR_ARG
    assert lib.gb_rotz_only(0, None, None) == L.GB_OK


def test_total_pixels_must_stay_below_2_31():
    """Packed pixel indices are int32 on the device: views whose pixels add up to 2^31 or more
    are refused on the host (three 32767 x 32767 views hold 3.2e9 pixels)."""
    big = [sg.look_at_view((0, 0, -3), 32767, 32767) for _ in range(3)]
    st, _ = _layout(P=10, views=big, cap=0)
    assert st == L.GB_ERR_ARG
    assert b"2^31" in _lib().gb_last_error()
    one_pass = L.make_options(prefix_pairs_per_tile=-1)  # (the prefix slots would not fit)
    assert _layout(P=10, views=big[:2], opts=one_pass, cap=0)[0] == L.GB_OK  # 2.1e9 < 2^31


def test_read_status_rejects_null_and_misaligned_arguments():
    lib = _lib()
    K = ctypes.c_int64(0)
    ov = ctypes.c_int32(0)
    assert lib.gb_read_status(None, ctypes.byref(K), ctypes.byref(ov), None, 1, None) == L.GB_ERR_ARG
    buf = ctypes.create_string_buffer(1024)
    base = ctypes.addressof(buf)
    p256 = base + (-base) % 256
    assert lib.gb_read_status(p256 + 4, ctypes.byref(K), ctypes.byref(ov), None, 1,
                              None) == L.GB_ERR_ARG
    assert lib.gb_read_status(p256, None, ctypes.byref(ov), None, 1, None) == L.GB_ERR_ARG


def test_densify_entry_points_check_arguments_before_any_launch():
    lib = _lib()
    assert lib.gb_densify_work_bytes(1000) >= 4 * 5 * 1000
    assert lib.gb_densify_work_bytes(-1) == 0
    o = L.GbDensifyOptions(2e-4, 0.01, 0.005, 0.0, 1.6)
    P = ctypes.c_int64(0)
    buf = ctypes.create_string_buffer(1 << 16)
    base = ctypes.addressof(buf)
    p256 = base + (-base) % 256
    raw = L.GbRawSplats(10, 4, 0, p256, p256, p256, p256, p256, None)
    assert lib.gb_densify_plan(None, p256, p256, ctypes.byref(o), p256, 1 << 15,
                               ctypes.byref(P), None) == L.GB_ERR_ARG
    bad = L.GbDensifyOptions(2e-4, 0.01, 0.005, 0.0, 0.5)  # split_shrink < 1
    assert lib.gb_densify_plan(ctypes.byref(raw), p256, p256, ctypes.byref(bad), p256, 1 << 15,
                               ctypes.byref(P), None) == L.GB_ERR_ARG
    assert lib.gb_densify_plan(ctypes.byref(raw), p256, p256, ctypes.byref(o), p256, 16,
                               ctypes.byref(P), None) == L.GB_ERR_ARG  # work buffer too small
    empty = L.GbRawSplats(0, 4, 0, None, None, None, None, None, None)
    assert lib.gb_densify_plan(ctypes.byref(empty), None, None, ctypes.byref(o), p256, 1 << 15,
                               ctypes.byref(P), None) == L.GB_OK and P.value == 0
    big = L.GbRawSplats(21, 4, 0, p256, p256, p256, p256, p256, None)
    assert lib.gb_densify_apply(ctypes.byref(raw), p256, p256, 0.5, ctypes.byref(o),
                                ctypes.byref(big), None, 0, None) == L.GB_ERR_ARG
    other_n = L.GbRawSplats(10, 8, 0, p256, p256, p256, p256, p256, None)
    assert lib.gb_densify_apply(ctypes.byref(raw), p256, p256, 0.5, ctypes.byref(o),
                                ctypes.byref(other_n), None, 0, None) == L.GB_ERR_ARG
    # the allocation-free variant: the same checks, and its size limit, before any launch
    dst = L.GbRawSplats(20, 4, 0, p256, p256, p256, p256, p256, None)
    assert lib.gb_densify_noalloc(None, p256, p256, ctypes.byref(o), p256, 0.5, ctypes.byref(dst),
                                  None, 0, ctypes.byref(P), None) == L.GB_ERR_ARG
    assert lib.gb_densify_noalloc(ctypes.byref(raw), p256, p256, ctypes.byref(bad), p256, 0.5,
                                  ctypes.byref(dst), None, 0, ctypes.byref(P), None) == L.GB_ERR_ARG
    assert lib.gb_densify_noalloc(ctypes.byref(raw), p256, p256, ctypes.byref(o), p256, 0.5,
                                  ctypes.byref(other_n), None, 0, ctypes.byref(P),
                                  None) == L.GB_ERR_ARG
    huge = L.GbRawSplats(L.DENSIFY_NOALLOC_MAX_P + 1, 4, 0, p256, p256, p256, p256, p256, None)
    assert lib.gb_densify_noalloc(ctypes.byref(huge), p256, p256, ctypes.byref(o), p256, 0.5,
                                  ctypes.byref(dst), None, 0, ctypes.byref(P),
                                  None) == L.GB_ERR_ARG
    assert b"GB_DENSIFY_NOALLOC_MAX_P" in lib.gb_last_error()
    empty_dst = L.GbRawSplats(0, 4, 0, None, None, None, None, None, None)
    P.value = 7
    assert lib.gb_densify_noalloc(ctypes.byref(empty), None, None, ctypes.byref(o), None, 0.5,
                                  ctypes.byref(empty_dst), None, 0, ctypes.byref(P),
                                  None) == L.GB_OK and P.value == 0
