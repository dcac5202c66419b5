"""The C-ABI library loads and exports every entry point include/hr.h declares
(no compute calls: these run without a GPU)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "hr.h")).read()
    return set(re.findall(r"^hr_status\s+(hr_\w+)\s*\(", src, flags=re.M))


def test_header_declares_entry_points():
    names = declared_entry_points()
    assert {"hr_ctx_create", "hr_shadow_alloc", "hr_kernel_end", "hr_report"} <= names


def test_library_exports_every_declared_symbol():
    from paper_2401_04701_amd import hr
    lib = hr.lib()
    names = declared_entry_points()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(hr.EXPORTED)


def test_binding_has_no_fallback_path():
    """The binding imports only libhr.so; it never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_2401_04701_amd", "hr.py")).read()
    assert "oracle" not in src


def test_unknown_config_flags_are_rejected():
    """Argument checks that run before any device call."""
    import ctypes
    from paper_2401_04701_amd import hr
    c = ctypes.c_void_p(0)
    cfg = hr._Config(0, 0, 0, 1 << 7, 0)
    assert hr.lib().hr_ctx_create(ctypes.byref(c), ctypes.byref(cfg), None) == hr.HR_E_INVAL
    cfg = hr._Config(0, 9, 0, 0, 0)                  # block clock wider than 8 bits
    assert hr.lib().hr_ctx_create(ctypes.byref(c), ctypes.byref(cfg), None) == hr.HR_E_INVAL
    # 4-byte words: a thread field above 10 bits
    cfg = hr._Config(0, 0, 0, hr.HR_CFG_WORD4, 0, 0, 0, 11)
    assert hr.lib().hr_ctx_create(ctypes.byref(c), ctypes.byref(cfg), None) == hr.HR_E_INVAL
    cfg = hr._Config(0, 0, 0, 0, 0, 0, 0, 8)         # a thread width without 4-byte words
    assert hr.lib().hr_ctx_create(ctypes.byref(c), ctypes.byref(cfg), None) == hr.HR_E_INVAL
    # coalescing widths: a power of two in 2..64, and only with wave grouping
    for width, flags in ((3, hr.HR_CFG_WAVE_GROUPING), (128, hr.HR_CFG_WAVE_GROUPING),
                         (1, hr.HR_CFG_WAVE_GROUPING), (16, 0)):
        cfg = hr._Config(0, 0, 0, flags, 0, 0, 0, 0, width)
        assert hr.lib().hr_ctx_create(ctypes.byref(c), ctypes.byref(cfg), None) == hr.HR_E_INVAL
    assert not c.value


def test_binding_site_ids_match_header():
    import re
    from paper_2401_04701_amd import hr
    text = open(os.path.join(ROOT, "include", "hr.h")).read()
    declared = {m.group(1): int(m.group(2))
                for m in re.finditer(r"\b(HR_SITE_[A-Z_]+) = (\d+)", text)}
    assert declared == hr.SITES
    assert "#define HR_SITES %d" % hr.HR_SITES in text

