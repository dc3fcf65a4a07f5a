"""Host-side checks of the C ABI with the real libp2o.so (no GPU needed):
every declared symbol is exported, argument and state checks return the
documented status without touching a device, and layout arithmetic matches
the header's contract."""
import ctypes
import os
import re
from ctypes import byref, c_int64, c_size_t, c_void_p

import pytest

from conftest import ROOT, ensure_built, gpu_available

ensure_built()
import paper_2501_14911_amd as p2o  # noqa: E402
from paper_2501_14911_amd._lib import lib  # noqa: E402

HEADER = os.path.join(ROOT, "include", "p2o.h")
OK, ARG, STATE, DTYPE, STORAGE, NONFINITE, HIP, NODEV = 0, -1, -2, -3, -4, -5, -6, -7


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(p2o_[a-zA-Z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14, names
    raw = ctypes.CDLL(p2o.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), f"{n} declared in p2o.h but not exported"


def create(Nd=600, Nm=16384, Nt=420, prec=2, max_rhs=1):
    plan = c_void_p()
    st = lib.p2o_create(byref(plan), Nd, Nm, Nt, prec, max_rhs)
    return st, plan


def test_status_strings():
    for code, name in [(OK, "P2O_OK"), (ARG, "P2O_ERR_ARG"), (STATE, "P2O_ERR_STATE"), (DTYPE, "P2O_ERR_DTYPE"),
                       (STORAGE, "P2O_ERR_STORAGE"), (NONFINITE, "P2O_ERR_NONFINITE"), (HIP, "P2O_ERR_HIP"),
                       (NODEV, "P2O_ERR_NO_DEVICE")]:
        assert p2o.status_name(code) == name
    assert p2o.status_name(12345) == "P2O_UNKNOWN_STATUS"


@pytest.mark.parametrize("args,code", [
    ((0, 10, 10, 0, 1), ARG), ((4, 0, 10, 0, 1), ARG), ((4, 10, 0, 0, 1), ARG),
    ((4, 10, 10, 0, 0), ARG), ((4, 10, 10, 7, 1), DTYPE), ((4, 10, 10, -1, 1), DTYPE),
    ((4, 10, 100000, 0, 1), ARG),
])
def test_create_rejects_bad_arguments(args, code):
    st, plan = create(*args)
    assert st == code
    assert p2o.last_error() != ""
    assert not plan.value


def test_create_null_out():
    assert lib.p2o_create(None, 4, 4, 4, 0, 1) == ARG


@pytest.mark.parametrize("Nt,L", [(1, 2), (2, 4), (13, 28), (16, 32), (21, 42), (128, 256), (420, 840), (500, 1000),
                                  (419, 840), (11, 24)])
def test_transform_length_is_twice_7smooth(Nt, L):
    st, plan = create(Nd=3, Nm=5, Nt=Nt, prec=0)
    assert st == OK
    Lv, nf, pitch, nblk = c_int64(), c_int64(), c_int64(), c_int64()
    assert lib.p2o_get_layout(plan, byref(Lv), byref(nf), byref(pitch), byref(nblk)) == OK
    assert Lv.value == L and nf.value == L // 2 + 1 and Lv.value >= 2 * Nt - 1
    assert pitch.value == 32 and nblk.value == 1
    lib.p2o_destroy(plan)


@pytest.mark.parametrize("Nm,pitch", [(1, 32), (32, 32), (33, 96), (1003, 1056), (16384, 16416), (16416, 16416),
                                      (16417, 16480), (65536, 65568)])
def test_spectrum_rows_start_an_odd_number_of_lines_apart(Nm, pitch):
    st, plan = create(Nd=3, Nm=Nm, Nt=16, prec=2)
    assert st == OK
    p = c_int64()
    assert lib.p2o_get_layout(plan, None, None, byref(p), None) == OK
    assert p.value == pitch and p.value >= Nm and p.value % 64 == 32
    lib.p2o_destroy(plan)


@pytest.mark.parametrize("prec,elem", [(0, 16), (1, 8), (2, 4), (3, 4)])
def test_required_bytes_cover_the_spectrum(prec, elem):
    st, plan = create(Nd=600, Nm=16384, Nt=420, prec=prec)
    assert st == OK
    fb, wb = c_size_t(), c_size_t()
    assert lib.p2o_required_bytes(plan, byref(fb), byref(wb)) == OK
    spec = 421 * 600 * 16416 * elem            # pitch 16416: the smallest >= 16384 that is 32 mod 64
    assert spec <= fb.value <= spec + 421 * 4 * 4 + 840 * 24 + 4096
    # workspace: one spectrum of the parameter series at least
    assert wb.value >= 421 * 16384 * (16 if prec == 0 else 8)
    lib.p2o_destroy(plan)


def test_bind_checks():
    st, plan = create(Nd=4, Nm=64, Nt=16, prec=0)
    fb, wb = c_size_t(), c_size_t()
    lib.p2o_required_bytes(plan, byref(fb), byref(wb))
    assert lib.p2o_bind_storage(plan, None, fb.value, c_void_p(4096), wb.value) == ARG
    assert lib.p2o_bind_storage(plan, c_void_p(4096 + 8), fb.value, c_void_p(8192), wb.value) == ARG
    assert lib.p2o_bind_storage(plan, c_void_p(4096), fb.value - 1, c_void_p(8192), wb.value) == STORAGE
    st = lib.p2o_bind_storage(plan, c_void_p(4096), fb.value, c_void_p(8192), wb.value)
    # host addresses: no device here, or not device memory on a GPU host
    assert st == (ARG if gpu_available() else NODEV)
    lib.p2o_destroy(plan)


def test_calls_out_of_order_and_bad_arguments():
    st, plan = create(Nd=4, Nm=64, Nt=16, prec=2, max_rhs=2)
    dummy = c_void_p(4096)
    assert lib.p2o_load_blocks(plan, dummy, 0, 64, 0) == STATE          # not bound
    assert lib.p2o_load_blocks(plan, dummy, 0, 64, 9) == DTYPE
    assert lib.p2o_load_blocks(plan, dummy, 0, 65, 0) == ARG
    assert lib.p2o_load_blocks(plan, None, 0, 64, 0) == ARG
    assert lib.p2o_load_finalize(plan) == STATE
    assert lib.p2o_apply_F(plan, dummy, dummy, 1, None) == STATE
    assert lib.p2o_apply_Ft(plan, dummy, dummy, 1, None) == STATE
    assert lib.p2o_apply_FFt(plan, dummy, dummy, 1, None) == STATE
    assert lib.p2o_apply_F(plan, dummy, dummy, 3, None) == ARG          # nrhs > max_rhs
    assert lib.p2o_apply_F(plan, dummy, dummy, 0, None) == ARG
    assert lib.p2o_apply_F(plan, None, dummy, 1, None) == ARG
    assert lib.p2o_apply_F(None, dummy, dummy, 1, None) == ARG
    assert lib.p2o_misfit_grad(plan, dummy, dummy, dummy, 5, dummy, dummy, 1, None) == ARG   # var length
    assert "noise_var_len" in p2o.last_error()
    assert lib.p2o_misfit_grad(plan, dummy, dummy, dummy, 4, dummy, dummy, 1, None) == STATE
    assert lib.p2o_misfit_grad(plan, dummy, None, dummy, 4, dummy, dummy, 1, None) == ARG
    assert lib.p2o_set_stream(plan, None) == OK
    assert lib.p2o_destroy(plan) == OK
    assert lib.p2o_destroy(None) == ARG


def test_scaled_loads_need_whole_blocks():
    st, plan = create(Nd=2, Nm=9000, Nt=8, prec=3)
    dummy = c_void_p(4096)
    assert lib.p2o_load_blocks(plan, dummy, 100, 4096, 0) == ARG
    assert lib.p2o_load_blocks(plan, dummy, 0, 1000, 0) == ARG
    assert "scale blocks" in p2o.last_error()
    # whole blocks and the ragged last block pass the argument checks (then fail on state)
    assert lib.p2o_load_blocks(plan, dummy, 0, 4096, 0) == STATE
    assert lib.p2o_load_blocks(plan, dummy, 8192, 808, 0) == STATE
    lib.p2o_destroy(plan)


def test_python_operator_requires_a_gpu_device():
    with pytest.raises(ValueError):
        p2o.P2OOperator(4, 64, 16, "fp64", device="cpu")


def test_gemm_tile_table_and_autotune_checks():
    tiles = p2o.gemm_tiles()
    assert tiles == [(2, 4, 5, 64), (2, 2, 5, 64), (4, 2, 5, 32), (2, 2, 4, 64), (4, 2, 4, 32), (2, 2, 5, 64),
                     (4, 2, 5, 64), (4, 2, 5, 64), (4, 2, 5, 32), (2, 2, 4, 64), (4, 2, 4, 32), (2, 2, 1, 64),
                     (4, 2, 1, 64), (2, 4, 5, 64), (2, 4, 5, 32), (4, 2, 4, 64), (2, 2, 4, 32), (2, 4, 1, 64),
                     (4, 4, 1, 64)]
    assert lib.p2o_gemm_tile_info(len(tiles), None, None, None, None) == ARG
    assert lib.p2o_gemm_tile_info(-1, None, None, None, None) == ARG
    st, plan = create(Nd=4, Nm=64, Nt=16, prec=2, max_rhs=4)
    assert lib.p2o_set_option(plan, 1, len(tiles)) == ARG
    assert lib.p2o_set_option(plan, 1, -2) == ARG
    assert lib.p2o_set_option(plan, 1, 0) == OK
    assert lib.p2o_set_option(plan, 1, -1) == OK
    assert lib.p2o_autotune(plan, 2, 3, None, None, None, None) == STATE      # not loaded
    assert lib.p2o_autotune(None, 2, 3, None, None, None, None) == ARG
    lib.p2o_destroy(plan)


def test_matrix_core_option_needs_a_16_bit_spectrum():
    """P2O_BATCHED_MFMA is accepted for BF16 and FP16 spectra (FP16 spectra take
    FP16 products with scaled FP16 right-hand sides) and refused for FP32 / FP64."""
    for prec, want in ((0, DTYPE), (1, DTYPE), (2, OK), (3, OK)):
        st, plan = create(Nd=4, Nm=64, Nt=16, prec=prec, max_rhs=4)
        assert st == OK
        assert lib.p2o_set_option(plan, 0, 2) == want, prec
        assert lib.p2o_set_option(plan, 0, 1) == OK
        assert lib.p2o_set_option(plan, 0, 3) == ARG
        lib.p2o_destroy(plan)


def test_fixed_length_fft_switch():
    st, plan = create(Nd=4, Nm=64, Nt=420, prec=1, max_rhs=2)
    assert st == OK
    for v in (0, 1):
        assert lib.p2o_set_option(plan, 2, v) == OK
    for v in (-1, 2):
        assert lib.p2o_set_option(plan, 2, v) == ARG
    assert lib.p2o_set_option(plan, 3, 0) == ARG          # output stride 0
    assert lib.p2o_set_option(plan, 99, 0) == ARG         # no such option
    lib.p2o_destroy(plan)


def test_fp16_operand_switch():
    """P2O_OPT_FP16_OPERANDS takes 0 or 1 on any plan (it only acts on FP16
    plans whose products run on the matrix cores)."""
    for prec in (0, 3):
        st, plan = create(Nd=4, Nm=64, Nt=420, prec=prec, max_rhs=2)
        assert st == OK
        for v in (0, 1):
            assert lib.p2o_set_option(plan, 4, v) == OK
        for v in (-1, 2):
            assert lib.p2o_set_option(plan, 4, v) == ARG
        lib.p2o_destroy(plan)


def test_bandwidth_probe_argument_checks():
    fake = c_void_p(1 << 20)                    # aligned, never dereferenced: every call fails before a launch
    assert lib.p2o_bandwidth_probe(0, fake, fake, 1024, 8, None) == ARG    # read probe: whole 2 KB chunks
    assert lib.p2o_bandwidth_probe(1, fake, fake, 48, 8, None) == ARG      # copy probe: multiples of 32
    assert lib.p2o_bandwidth_probe(2, fake, fake, 2048, 8, None) == ARG
    assert lib.p2o_bandwidth_probe(0, fake, fake, 2048, 0, None) == ARG
    assert lib.p2o_bandwidth_probe(0, None, fake, 2048, 8, None) == ARG
