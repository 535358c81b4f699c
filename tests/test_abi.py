"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/ccl.h declares, and rejects invalid arguments with the
documented status before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1708_08180_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(ccl_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    names = declared_symbols()
    assert "ccl_label_2d" in names
    for n in sorted(names):
        assert hasattr(lib, n), "libccl.so does not export %s" % n
        assert n in binding.SIGNATURES, "binding has no signature for %s" % n


def test_status_strings_and_version():
    lib = binding.load_library()
    for code in range(0, 8):
        assert lib.ccl_status_string(code)
    assert lib.ccl_status_string(99) == b"unknown ccl status"
    assert lib.ccl_version() >= 10000


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
LAB = ctypes.c_void_p(1 << 40)  # a label buffer far from FAKE (no overlap)


@pytest.mark.parametrize("args,code", [
    ((None, 4, 4, 4, 8, LAB, None), 1),        # null image
    ((FAKE, 4, 4, 4, 8, None, None), 1),        # null labels
    ((FAKE, 0, 4, 4, 8, LAB, None), 1),        # H = 0
    ((FAKE, 4, -1, 4, 8, LAB, None), 1),       # W < 0
    ((FAKE, 4, 8, 7, 8, LAB, None), 1),        # pitch < W
    ((FAKE, 4, 4, 4, 6, LAB, None), 2),        # connectivity 6
    ((FAKE, 65536, 65537, 65537, 8, LAB, None), 3),  # H*W > 2^32-1
])
def test_invalid_arguments(args, code):
    lib = binding.load_library()
    assert lib.ccl_label_2d(*args) == code


@pytest.mark.parametrize("args,code", [
    ((None, 4, 4, 4, 8, LAB, None, None), 1),        # null image
    ((FAKE, 4, 4, 4, 8, None, None, None), 1),        # null labels
    ((FAKE, 4, 8, 7, 8, LAB, None, None), 1),        # pitch < W
    ((FAKE, 4, 4, 4, 6, LAB, None, None), 2),        # connectivity 6
    ((FAKE, 65536, 65537, 65537, 8, LAB, None, None), 3),  # H*W > 2^32-1
])
def test_equal_invalid_arguments(args, code):
    lib = binding.load_library()
    assert lib.ccl_label_2d_equal(*args) == code


def test_equal_config_validation():
    # only (16,4) (32,2) (32,8) (64,4) (64,8) are compiled for equal-value labeling
    lib = binding.load_library()
    for th, nw in ((64, 1), (64, 16), (16, 1), (48, 4)):
        cfg = binding.Config(th, nw)
        assert lib.ccl_label_2d_equal(FAKE, 64, 64, 64, 8, LAB, ctypes.byref(cfg), None) == 2


@pytest.mark.parametrize("args,code", [
    ((None, 2, 4, 4, 4, 16, 26, LAB, None), 1),          # null volume
    ((FAKE, 0, 4, 4, 4, 16, 26, LAB, None), 1),          # D = 0
    ((FAKE, 2, 4, 8, 7, 32, 26, LAB, None), 1),          # pitch_y < W
    ((FAKE, 2, 4, 8, 8, 31, 26, LAB, None), 1),          # pitch_z < H * pitch_y
    ((FAKE, 2, 4, 4, 4, 16, 8, LAB, None), 2),           # connectivity 8
    ((FAKE, 2048, 2048, 2048, 2048, 2048 * 2048, 6, LAB, None), 3),  # D*H*W > 2^32-1
])
def test_3d_invalid_arguments(args, code):
    lib = binding.load_library()
    assert lib.ccl_label_3d(*args) == code


def test_ex_validation():
    lib = binding.load_library()
    cfg = binding.Config(48, 4)
    assert lib.ccl_label_2d_ex(FAKE, 64, 64, 64, 8, LAB, None, 0, ctypes.byref(cfg), None) == 2
    cfg = binding.Config(64, 3)
    assert lib.ccl_label_2d_ex(FAKE, 64, 64, 64, 8, LAB, None, 0, ctypes.byref(cfg), None) == 2
    # caller workspace too small / misaligned
    assert lib.ccl_label_2d_ex(FAKE, 64, 64, 64, 8, LAB, FAKE, 16, None, None) == 7
    big = binding.workspace_size(64, 64)
    odd = ctypes.c_void_p(0x1001)
    assert lib.ccl_label_2d_ex(FAKE, 64, 64, 64, 8, LAB, odd, big, None, None) == 1


def test_workspace_size_formula():
    # per tile: 4 edge masks (8 B), 2*64 + 2*TH edge roots (4 B), 2*TH row
    # masks (8 B: foreground, edge roots), TH/2 band interval-end masks (8 B),
    # TH/2 two-byte band bases and 32 two-byte records per row; each part
    # 256-byte aligned
    for (H, W, th) in ((4096, 4096, 64), (100, 65, 16), (1, 1, 32)):
        tiles = (-(-W // 64)) * (-(-H // th))
        masks = -(-tiles * 32 // 256) * 256
        roots = -(-tiles * (128 + 2 * th) * 4 // 256) * 256
        rowm = -(-tiles * (2 * th + th // 2 + th // 8) * 8 // 256) * 256
        slots = -(-tiles * th * 64 // 256) * 256
        assert binding.workspace_size(H, W, (th, 4 if th >= 4 else 1)) == masks + roots + rowm + slots


def test_batch_validation_without_device():
    lib = binding.load_library()
    h = ctypes.c_void_p()
    assert lib.ccl_ctx_create(None, None) == 1
    opts = binding.CtxOpts(0, 100, binding.Config(0, 0), 1)
    assert lib.ccl_ctx_create(ctypes.byref(h), ctypes.byref(opts)) == 1   # max_images < 1
    opts = binding.CtxOpts(4, 0, binding.Config(0, 0), 1)
    assert lib.ccl_ctx_create(ctypes.byref(h), ctypes.byref(opts)) == 1   # max_pixels < 1
    assert lib.ccl_label_batch(None, None, 1, 8, None) == 1
    assert lib.ccl_ctx_destroy(None) == 1


def test_autotune_validation_without_device():
    lib = binding.load_library()
    best = binding.Config(0, 0)
    assert lib.ccl_autotune(None, 8, 8, 8, 8, FAKE, 3, None, ctypes.byref(best), None) == 1
    assert lib.ccl_autotune(FAKE, 8, 8, 8, 5, LAB, 3, None, ctypes.byref(best), None) == 2
    assert lib.ccl_autotune(FAKE, 8, 8, 8, 8, LAB, 0, None, ctypes.byref(best), None) == 1


def test_tuning_table_roundtrip(tmp_path):
    binding.tuning_clear()
    assert binding.tuning_get(4096, 4096, 8) == (64, 4)       # built-in default, large images
    assert binding.tuning_get(1080, 1920, 8) == (32, 4)       # built-in default, below 2^22 px
    src = tmp_path / "in.jsonl"
    src.write_text('{"class": 24, "conn": 8, "tile_h": 32, "waves": 2, "ms": 0.150000}\n'
                   '{"class": 20, "conn": 4, "tile_h": 16, "waves": 1, "ms": 0.020000}\n')
    binding.tuning_load(str(src))
    assert binding.tuning_get(4096, 4096, 8) == (32, 2)       # 2^24 pixels -> class 24
    assert binding.tuning_get(4096, 4096, 4) == (64, 4)       # other connectivity: default
    assert binding.tuning_get(1024, 1024, 4) == (16, 1)       # 2^20 pixels -> class 20
    out = tmp_path / "out.jsonl"
    binding.tuning_save(str(out))
    lines = sorted(out.read_text().strip().splitlines())
    assert len(lines) == 2 and '"tile_h": 32' in "".join(lines)
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"class": 24, "conn": 8, "tile_h": 48, "waves": 4, "ms": 1.0}\n')
    with pytest.raises(binding.CclError):
        binding.tuning_load(str(bad))
    binding.tuning_clear()
    assert binding.tuning_get(4096, 4096, 8) == (64, 4)


@pytest.mark.parametrize("args,code", [
    ((None, 4, 4, 4, 8, LAB, None), 1),        # null image
    ((FAKE, 4, 4, 4, 8, None, None), 1),        # null labels
    ((FAKE, 0, 4, 4, 8, LAB, None), 1),        # H = 0
    ((FAKE, 4, 8, 7, 8, LAB, None), 1),        # pitch < W
    ((FAKE, 4, 4, 4, 6, LAB, None), 2),        # connectivity 6
    ((FAKE, 65536, 65537, 65537, 8, LAB, None), 3),  # H*W > 2^32-1
    ((FAKE, 8192, 8192, 8192, 8, LAB, None), 7),     # needs more than the fixed array
    ((FAKE, 1, 60000000, 60000000, 4, LAB, None), 7),
])
def test_noalloc_invalid_arguments(args, code):
    """The fixed-workspace entry point rejects bad arguments, and images
    whose workspace exceeds its array, before any HIP call."""
    lib = binding.load_library()
    assert lib.ccl_label_2d_noalloc(*args) == code


def test_noalloc_limit_covers_4096_square():
    lib = binding.load_library()
    size = ctypes.c_size_t(0)
    assert lib.ccl_workspace_size(4096, 4096, None, ctypes.byref(size)) == 0
    limit = 32 << 20
    assert 0 < size.value <= limit
    assert lib.ccl_workspace_size(8192, 8192, None, ctypes.byref(size)) == 0
    assert size.value > limit


def test_ctx_autotune_validation_without_device():
    lib = binding.load_library()
    cfg = binding.Config()
    assert lib.ccl_ctx_config(None, 8, ctypes.byref(cfg)) == 1
    assert lib.ccl_ctx_autotune(None, None, 1, 8, 1, None, None, None) == 1


@pytest.mark.parametrize("args,code", [
    ((None, 4, 4, 4, 8, LAB, FAKE, 1, FAKE, None, None), 1),      # null image
    ((FAKE, 4, 4, 4, 8, None, FAKE, 1, FAKE, None, None), 1),      # null labels
    ((FAKE, 4, 4, 4, 8, LAB, FAKE, 1, None, None, None), 1),      # null count
    ((FAKE, 4, 4, 4, 8, LAB, None, 1, FAKE, None, None), 1),      # capacity without records
    ((FAKE, 4, 4, 4, 8, LAB, FAKE, -1, FAKE, None, None), 1),     # capacity < 0
    ((FAKE, 4, 8, 7, 8, LAB, FAKE, 1, FAKE, None, None), 1),      # pitch < W
    ((FAKE, 4, 4, 4, 6, LAB, FAKE, 1, FAKE, None, None), 2),      # connectivity 6
    ((FAKE, 65536, 65537, 65537, 8, LAB, FAKE, 1, FAKE, None, None), 3),  # H*W > 2^32-1
])
def test_label_stats_invalid_arguments(args, code):
    """The labels-with-statistics entry point validates like ccl_label_2d
    and ccl_component_stats, before touching the device."""
    lib = binding.load_library()
    assert lib.ccl_label_2d_stats(*args) == code


def test_label_stats_config_validation():
    # tiles of more than 64 rows, and configurations not compiled at all
    lib = binding.load_library()
    for th, nw in ((128, 4), (128, 8), (48, 4), (64, 3)):
        cfg = binding.Config(th, nw)
        assert lib.ccl_label_2d_stats(FAKE, 64, 64, 64, 8, LAB, FAKE, 1, FAKE, ctypes.byref(cfg), None) == 2


def test_overlapping_image_and_labels_are_rejected():
    """Image and label bytes that intersect are an invalid argument, for
    every entry point that takes both; adjacent buffers are fine."""
    lib = binding.load_library()
    img = 0x100000
    H, W, pitch = 16, 20, 32
    end = img + (H - 1) * pitch + W                     # one past the image's last byte
    inside = ctypes.c_void_p(img + 8)
    assert lib.ccl_label_2d(ctypes.c_void_p(img), H, W, pitch, 8, inside, None) == 1
    assert lib.ccl_label_2d(ctypes.c_void_p(img), H, W, pitch, 8, ctypes.c_void_p(end - 1), None) == 1
    below = ctypes.c_void_p(img - H * W * 4 + 4)        # labels ending inside the image
    assert lib.ccl_label_2d(ctypes.c_void_p(img), H, W, pitch, 8, below, None) == 1
    # adjacent on either side: validation passes (connectivity 6 is the error)
    assert lib.ccl_label_2d(ctypes.c_void_p(img), H, W, pitch, 6, ctypes.c_void_p(end), None) == 2
    assert lib.ccl_label_2d(ctypes.c_void_p(img), H, W, pitch, 6, ctypes.c_void_p(img - H * W * 4), None) == 2
    assert lib.ccl_label_2d_equal(ctypes.c_void_p(img), H, W, pitch, 8, inside, None, None) == 1
    assert lib.ccl_label_2d_ex(ctypes.c_void_p(img), H, W, pitch, 8, inside, None, 0, None, None) == 1
    assert lib.ccl_label_2d_noalloc(ctypes.c_void_p(img), H, W, pitch, 8, inside, None) == 1
    assert lib.ccl_label_2d_stats(ctypes.c_void_p(img), H, W, pitch, 8, inside, LAB, 1, FAKE, None, None) == 1
    # a volume: D slices of H rows
    D, py, pz = 3, 32, 16 * 32
    vend = img + (D - 1) * pz + (H - 1) * py + W
    assert lib.ccl_label_3d(ctypes.c_void_p(img), D, H, W, py, pz, 26, ctypes.c_void_p(vend - 4), None) == 1
    assert lib.ccl_label_3d(ctypes.c_void_p(img), D, H, W, py, pz, 8, ctypes.c_void_p(vend), None) == 2
