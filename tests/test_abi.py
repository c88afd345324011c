"""Host-only checks of the C ABI: the built library loads and exports every function the header
declares, and argument validation that happens before any device work returns the documented
status codes (no GPU needed)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dtrg.h")
LIB = os.path.join(ROOT, "paper_1912_02780_amd", "libdtrg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(dtrg_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("libdtrg.so not built (run python -m paper_1912_02780_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dtrg_hotrg_forward", "dtrg_hotrg_backward", "dtrg_plan_step_info", "dtrg_plan_destroy",
                     "dtrg_last_error", "dtrg_default_options"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    src = open(os.path.join(ROOT, "paper_1912_02780_amd", "binding.py")).read()
    m = re.search(r"EXPORTED = \[(.*?)\]", src, flags=re.S)
    exported = sorted(re.findall(r'"(dtrg_[a-z0-9_]+)"', m.group(1)))
    assert exported == declared_functions()


def test_argument_validation_without_device_work():
    lib = _lib()
    lib.dtrg_hotrg_forward.restype = ctypes.c_int
    lib.dtrg_hotrg_backward.restype = ctypes.c_int
    lib.dtrg_plan_step_info.restype = ctypes.c_int
    lib.dtrg_last_error.restype = ctypes.c_char_p
    plan = ctypes.c_void_p()
    out = ctypes.c_double()
    # NULL T0 -> DTRG_EINVAL (1), plan set to NULL
    st = lib.dtrg_hotrg_forward(None, 2, 4, 3, None, None, ctypes.byref(plan), ctypes.byref(out))
    assert st == 1 and plan.value is None
    assert b"NULL" in lib.dtrg_last_error()
    # chi out of range with a non-NULL (never dereferenced) pointer
    st = lib.dtrg_hotrg_forward(ctypes.c_void_p(8), 2, 0, 3, None, None, ctypes.byref(plan), ctypes.byref(out))
    assert st == 1
    st = lib.dtrg_hotrg_forward(ctypes.c_void_p(8), 2, 4, 0, None, None, ctypes.byref(plan), ctypes.byref(out))
    assert st == 1
    # backward / step info on a NULL plan
    assert lib.dtrg_hotrg_backward(None, ctypes.c_double(1.0), ctypes.c_void_p(8), None, None, None) == 1
    assert lib.dtrg_plan_step_info(None, 1, None) == 1
    lib.dtrg_plan_destroy(None)
    # plan creation with bad sizes fails before any allocation
    lib.dtrg_plan_create.restype = ctypes.c_int
    assert lib.dtrg_plan_create(2, 0, 3, None, ctypes.byref(plan)) == 1 and plan.value is None
    assert lib.dtrg_plan_create(0, 4, 3, None, ctypes.byref(plan)) == 1
    lib.dtrg_plan_forward.restype = ctypes.c_int
    assert lib.dtrg_plan_forward(None, ctypes.c_void_p(8), None, ctypes.byref(out)) == 1


# the header's structs, field by field, as ctypes types (parsed from include/dtrg.h)
_CTYPES = {"int": ctypes.c_int, "double": ctypes.c_double, "const char*": ctypes.c_char_p,
           "dtrg_alloc_fn": ctypes.c_void_p, "dtrg_free_fn": ctypes.c_void_p, "void*": ctypes.c_void_p}


def header_struct(name):
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", src).group(1)
    fields = []
    for decl in body.split(";"):
        decl = " ".join(decl.split())
        if not decl:
            continue
        assert "," not in decl, "one field per declaration in " + name
        m = re.match(r"(.*?)\s*\b(\w+)$", decl)
        fields.append((m.group(2), _CTYPES[m.group(1).replace(" *", "*").strip()]))
    return fields


def _struct(name):
    return type(name, (ctypes.Structure,), {"_fields_": header_struct(name)})


def test_binding_structs_match_header():
    """Field names, order and C types of dtrg_options and dtrg_step_info in the binding are the header's."""
    torch = pytest.importorskip("torch")   # noqa: F841  (the binding imports it)
    if not os.path.exists(LIB):
        pytest.skip("libdtrg.so not built")
    from paper_1912_02780_amd import binding as B
    for name, cls in (("dtrg_options", B.Options), ("dtrg_step_info", B.StepInfo)):
        hdr = header_struct(name)
        assert [f for f, _ in cls._fields_] == [f for f, _ in hdr], name
        assert ctypes.sizeof(cls) == ctypes.sizeof(_struct(name)), name


def test_default_options():
    lib = _lib()
    Options = _struct("dtrg_options")
    o = Options()
    lib.dtrg_default_options(ctypes.byref(o))
    assert o.contract == 0 and o.eig_broadening == 1e-12 and o.max_subspace_iters == 60
    assert o.autotune == 0 and o.profile == 0 and o.gram_fp64 == 1 and o.checkpoint_gib == 64.0
    assert o.oversample == 0 and o.max_fp32_chain == 4096 and o.max_fp32_chain_wide == 4096
    assert o.tile_table is None and o.alloc_fn is None and o.free_fn is None
    assert o.chain_phys == 0 and o.side_rule == 0 and o.polar_newton == 0 and o.subspace_shift == 1 and o.rr_skip == 3
    # a checkpoint budget that is negative or not finite is rejected before any allocation
    lib.dtrg_plan_create.restype = ctypes.c_int
    lib.dtrg_last_error.restype = ctypes.c_char_p
    plan = ctypes.c_void_p()
    for bad in (-1.0, float("nan"), float("inf")):
        o.checkpoint_gib = bad
        assert lib.dtrg_plan_create(2, 4, 3, ctypes.byref(o), ctypes.byref(plan)) == 1 and plan.value is None
        assert b"checkpoint_gib" in lib.dtrg_last_error()


def test_side_rule_validation_without_device_work():
    lib = _lib()
    lib.dtrg_plan_create.restype = ctypes.c_int
    lib.dtrg_batch_create.restype = ctypes.c_int
    lib.dtrg_last_error.restype = ctypes.c_char_p
    Options = _struct("dtrg_options")
    plan = ctypes.c_void_p()
    for rule, phys, msg in ((2, 0, b"side_rule"), (-1, 0, b"side_rule"), (1, 2, b"scheme (a)")):
        o = Options()
        lib.dtrg_default_options(ctypes.byref(o))
        o.side_rule, o.chain_phys = rule, phys
        assert lib.dtrg_plan_create(2, 4, 3, ctypes.byref(o), ctypes.byref(plan)) == 1 and plan.value is None
        assert msg in lib.dtrg_last_error()
    o = Options()
    lib.dtrg_default_options(ctypes.byref(o))
    o.side_rule = 1
    b = ctypes.c_void_p()
    chis = (ctypes.c_int * 2)(8, 8)
    assert lib.dtrg_batch_create(2, 2, chis, 4, ctypes.byref(o), ctypes.byref(b)) == 1
    assert b"side_rule" in lib.dtrg_last_error() and b.value is None


def test_batch_argument_validation_without_device_work():
    lib = _lib()
    lib.dtrg_batch_create.restype = ctypes.c_int
    lib.dtrg_batch_run.restype = ctypes.c_int
    lib.dtrg_batch_step_info.restype = ctypes.c_int
    lib.dtrg_last_error.restype = ctypes.c_char_p
    b = ctypes.c_void_p()
    chis = (ctypes.c_int * 3)(16, 24, 0)
    # a chi out of range anywhere in the batch fails before any allocation
    assert lib.dtrg_batch_create(3, 2, chis, 30, None, ctypes.byref(b)) == 1 and b.value is None
    assert b"chi" in lib.dtrg_last_error()
    assert lib.dtrg_batch_create(0, 2, chis, 30, None, ctypes.byref(b)) == 1
    assert lib.dtrg_batch_create(2, 2, None, 30, None, ctypes.byref(b)) == 1
    assert lib.dtrg_batch_create(2, 2, chis, 0, None, ctypes.byref(b)) == 1
    out = (ctypes.c_double * 3)()
    assert lib.dtrg_batch_run(None, ctypes.c_void_p(8), None, ctypes.c_double(1.0), out, None, None, 0, None) == 1
    assert lib.dtrg_batch_step_info(None, 0, 1, None) == 1
    lib.dtrg_batch_destroy(None)
    lib.dtrg_batch_device_bytes.restype = ctypes.c_size_t
    assert lib.dtrg_batch_device_bytes(None) == 0


def test_contract_config_validation_without_device_work():
    """Bad tile codes and split counts are rejected before any device work (the pointers are never
    dereferenced)."""
    lib = _lib()
    f = lib.dtrg_contract_config
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong,
                  ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong,
                  ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    lib.dtrg_last_error.restype = ctypes.c_char_p
    p = ctypes.c_void_p(64)
    # FP64 and FP32 have tiles 1 and 2 only; the bf16-plane precisions 1 to 6; split counts 0 to 64
    for prec, tile, splits in ((0, 3, 0), (0, 6, 0), (1, 5, 0), (3, 7, 0), (3, -1, 0), (3, 1, 65), (0, 1, -1)):
        st = f(prec, 8, 8, 8, p, 8, 0, p, 8, 0, p, 8, 1, 1.0, 0.0, tile, splits, None)
        assert st == 1, (prec, tile, splits)
        msg = lib.dtrg_last_error()
        assert b"tile" in msg or b"split" in msg
    # tile 6: K-contiguous operands and K a multiple of 16 only
    for tile, K, akm, bkm in ((6, 20, 0, 0), (6, 8, 0, 0), (6, 32, 1, 0), (6, 32, 0, 1)):
        st = f(3, 8, 8, K, p, 64, akm, p, 64, bkm, p, 8, 1, 1.0, 0.0, tile, 1, None)
        assert st == 1, (tile, K, akm, bkm)
        assert b"tile" in lib.dtrg_last_error()
    # NULL operands and short leading dimensions are rejected first
    assert f(3, 8, 8, 8, None, 8, 0, p, 8, 0, p, 8, 1, 1.0, 0.0, 1, 1, None) == 1
    assert f(3, 8, 8, 8, p, 4, 0, p, 8, 0, p, 8, 1, 1.0, 0.0, 1, 1, None) == 1


# ---------------------------------------------------------------------------------------------
# plans on a caller's allocator that hands out addresses the library never dereferences before a
# forward pass: allocation failure, out-of-order calls and release, all without a GPU
# ---------------------------------------------------------------------------------------------
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class FakeDeviceMemory:
    """Hands out distinct 256-byte aligned addresses (never dereferenced) and records the frees."""

    def __init__(self, fail_after=None, align=256):
        self.live = {}
        self.next = 1 << 40
        self.allocs = 0
        self.fail_after = fail_after
        self.align = align
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, stream, user):
        if self.fail_after is not None and self.allocs >= self.fail_after:
            return None
        self.allocs += 1
        p = self.next + (self.align % 256)
        self.next += (nbytes + 4095) // 4096 * 4096 + 4096
        self.live[p] = nbytes
        return p

    def _free(self, ptr, nbytes, stream, user):
        assert self.live.pop(ptr) == nbytes


def _plan_create(lib, mem, **opt):
    Options = _struct("dtrg_options")
    o = Options()
    lib.dtrg_default_options(ctypes.byref(o))
    for k, v in opt.items():
        setattr(o, k, v)
    o.alloc_fn = ctypes.cast(mem.alloc_fn, ctypes.c_void_p) if mem else None
    o.free_fn = ctypes.cast(mem.free_fn, ctypes.c_void_p) if mem else None
    lib.dtrg_plan_create.restype = ctypes.c_int
    plan = ctypes.c_void_p()
    st = lib.dtrg_plan_create(2, 16, 12, ctypes.byref(o), ctypes.byref(plan))
    return st, plan


def test_allocator_failure_is_enomem_and_leaks_nothing():
    lib = _lib()
    lib.dtrg_last_error.restype = ctypes.c_char_p
    for fail_after in (0, 5, 40):
        mem = FakeDeviceMemory(fail_after=fail_after)
        st, plan = _plan_create(lib, mem)
        assert st == 2 and plan.value is None, (fail_after, st)      # DTRG_ENOMEM
        assert b"alloc_fn" in lib.dtrg_last_error()
        assert not mem.live, "blocks allocated before the failure must be released"


def test_backward_before_forward_is_estate_and_destroy_frees_every_block():
    lib = _lib()
    lib.dtrg_last_error.restype = ctypes.c_char_p
    lib.dtrg_hotrg_backward.restype = ctypes.c_int
    lib.dtrg_plan_step_info.restype = ctypes.c_int
    lib.dtrg_plan_device_bytes.restype = ctypes.c_size_t
    mem = FakeDeviceMemory()
    st, plan = _plan_create(lib, mem)
    assert st == 0 and plan.value
    assert mem.allocs > 10 and mem.live
    assert lib.dtrg_plan_device_bytes(plan) == sum(mem.live.values())
    # no forward yet: the backward and the diagnostics refuse before touching the device
    st = lib.dtrg_hotrg_backward(plan, ctypes.c_double(1.0), ctypes.c_void_p(1 << 40), None, None, None)
    assert st == 6 and b"before" in lib.dtrg_last_error()           # DTRG_ESTATE
    info = (ctypes.c_char * 256)()
    assert lib.dtrg_plan_step_info(plan, 1, info) == 6
    lib.dtrg_plan_destroy(plan)
    assert not mem.live


def test_allocator_callbacks_are_validated():
    lib = _lib()
    lib.dtrg_last_error.restype = ctypes.c_char_p
    mem = FakeDeviceMemory()
    Options = _struct("dtrg_options")
    o = Options()
    lib.dtrg_default_options(ctypes.byref(o))
    o.alloc_fn = ctypes.cast(mem.alloc_fn, ctypes.c_void_p)        # free_fn left NULL
    plan = ctypes.c_void_p()
    lib.dtrg_plan_create.restype = ctypes.c_int
    assert lib.dtrg_plan_create(2, 16, 12, ctypes.byref(o), ctypes.byref(plan)) == 1
    assert b"free_fn" in lib.dtrg_last_error() and mem.allocs == 0
    # an allocator that returns memory the kernels cannot use (not 256-byte aligned)
    bad = FakeDeviceMemory(align=8)
    st, plan = _plan_create(lib, bad)
    assert st == 1 and plan.value is None and b"aligned" in lib.dtrg_last_error()
    assert not bad.live


def test_option_ranges_are_validated():
    lib = _lib()
    lib.dtrg_last_error.restype = ctypes.c_char_p
    for field, value in (("max_fp32_chain", 16), ("max_fp32_chain_wide", 1 << 21), ("oversample", 96),
                         ("oversample", -1), ("subspace_shift", 2), ("subspace_shift", -1), ("rr_skip", 4),
                         ("rr_skip", -1), ("polar_newton", 2)):
        st, plan = _plan_create(lib, FakeDeviceMemory(), **{field: value})
        assert st == 1 and plan.value is None, field
        assert field.encode() in lib.dtrg_last_error()
