"""The C-ABI library loads on a machine without a GPU and exports every symbol
include/hap.h declares; argument checks that need no device answer correctly."""
import ctypes
import os
import re

import pytest

from paper_1403_7394_amd import hap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hap.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hap_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hap.LIB_PATH):
        pytest.fail("libhap.so is not built (run python -m paper_1403_7394_amd.build)")
    return hap.load()


def test_header_declares_the_binding_exports():
    assert _declared_functions() == sorted(hap.EXPORTS)


def _header_enums():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return {k: int(v) for k, v in re.findall(r"\b(HAP_[A-Z0-9_]+)\s*=\s*(\d+)", text)}


def test_binding_constants_equal_the_header_enums():
    """Every constant the binding passes or tests against has the header's value (the
    binding strips the HAP_ prefix of the launch, build, preference and schedule names)."""
    enums = _header_enums()
    checked = 0
    for name, value in enums.items():
        for attr in (name, name[len("HAP_"):]):
            if hasattr(hap, attr):
                assert getattr(hap, attr) == value, name
                checked += 1
                break
    for name in ("HAP_LAUNCH_STREAM", "HAP_LAUNCH_EAGER", "HAP_LAUNCH_UNFUSED", "HAP_LAUNCH_FUSED",
                 "HAP_LAUNCH_BLOCKS", "HAP_SCHEDULE_MRHAP", "HAP_BUILD_DIRECT_L2", "HAP_E_UNSUPPORTED"):
        assert name in enums, name
    assert checked >= 20, checked


def test_every_declared_symbol_is_exported(lib):
    missing = [name for name in _declared_functions() if not hasattr(lib, name)]
    assert not missing


def test_version_and_status_strings(lib):
    assert b"gfx950" in lib.hap_version()
    assert lib.hap_status_string(hap.HAP_OK) == b"ok"
    assert lib.hap_status_string(hap.HAP_E_ARG) == b"invalid argument"


def test_workspace_size_checks_arguments(lib):
    b = ctypes.c_size_t()
    assert lib.hap_workspace_size(1, 3, hap.HAP_F32, ctypes.byref(b)) == hap.HAP_E_ARG
    assert lib.hap_workspace_size(100, 0, hap.HAP_F32, ctypes.byref(b)) == hap.HAP_E_ARG
    assert lib.hap_workspace_size(100, 3, 7, ctypes.byref(b)) == hap.HAP_E_DTYPE
    assert lib.hap_workspace_size(100, 3, hap.HAP_F32, None) == hap.HAP_E_ARG
    assert lib.hap_workspace_size(8192, 3, hap.HAP_F32, ctypes.byref(b)) == hap.HAP_OK
    # two N x N message matrices per level dominate
    assert b.value >= 2 * 3 * 8192 * 8192 * 4
    assert b.value < 2 * 3 * 8192 * 8192 * 4 * 1.1


def test_init_rejects_bad_arguments_without_touching_the_device(lib):
    p = hap.hap_params()
    p.struct_size = ctypes.sizeof(hap.hap_params)
    p.levels = 3
    p.damping = 0.5
    p.pref_mode = hap.PREF_MEDIAN
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(4096)  # never dereferenced: every call below fails its checks first
    assert lib.hap_init(None, fake, 10, 12, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    assert lib.hap_init(ctypes.byref(ctx), fake, 1, 12, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    assert lib.hap_init(ctypes.byref(ctx), fake, 10, 9, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    assert lib.hap_init(ctypes.byref(ctx), fake, 10, 10, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    assert lib.hap_init(ctypes.byref(ctx), fake, 10, 12, 5, ctypes.byref(p), None, 0, None) == hap.HAP_E_DTYPE
    p.damping = 1.0
    assert lib.hap_init(ctypes.byref(ctx), fake, 10, 12, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    p.damping = 0.5
    p.levels = 0
    assert lib.hap_init(ctypes.byref(ctx), fake, 10, 12, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    p.levels = 2
    p.pref_mode = hap.PREF_SCALAR
    bad = (ctypes.c_double * 2)(1.0, float("nan"))
    p.pref_scalar = ctypes.cast(bad, ctypes.POINTER(ctypes.c_double))
    assert lib.hap_init(ctypes.byref(ctx), fake, 10, 12, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    assert b"non-finite" in lib.hap_last_error()
    p.pref_mode = hap.PREF_MEDIAN
    # Eq. 2.7 weight: in [0, 1], and only with the level-sequential schedule
    for kappa, schedule in [(1.5, hap.SCHEDULE_SEQUENTIAL), (-0.25, hap.SCHEDULE_SEQUENTIAL),
                            (float("nan"), hap.SCHEDULE_SEQUENTIAL), (0.5, hap.SCHEDULE_MRHAP)]:
        p.kappa, p.schedule = kappa, schedule
        assert lib.hap_init(ctypes.byref(ctx), fake, 10, 12, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
        assert b"kappa" in lib.hap_last_error()
    p.kappa, p.schedule = 0.0, hap.SCHEDULE_SEQUENTIAL
    p.struct_size = 8
    assert lib.hap_init(ctypes.byref(ctx), fake, 10, 12, hap.HAP_F32, ctypes.byref(p), None, 0, None) == hap.HAP_E_ARG
    assert not ctx.value


def test_null_context_calls_fail_cleanly(lib):
    out = ctypes.c_int32()
    assert lib.hap_iterate(None, 1, 0, ctypes.byref(out), None) == hap.HAP_E_ARG
    assert lib.hap_exemplars(None, 0, None, None) == hap.HAP_E_ARG
    assert lib.hap_similarity_offsets(None, 0, None) == hap.HAP_E_ARG
    assert lib.hap_destroy(None) == hap.HAP_OK
    d = ctypes.c_double()
    assert lib.hap_net_similarity(None, 0, None, 0, 0, 0, ctypes.byref(d)) == hap.HAP_E_ARG
    fake = ctypes.c_void_p(4096)
    assert lib.hap_set_points(None, fake, 100, 2, 2, hap.HAP_F32) == hap.HAP_E_ARG
    assert lib.hap_set_row_count(None, 10) == hap.HAP_E_ARG
    assert lib.hap_set_launch(None, 256, 1, 1, 0) == hap.HAP_E_ARG


def test_build_and_median_check_arguments(lib):
    fake = ctypes.c_void_p(4096)
    assert lib.hap_build_similarity(None, 10, 2, 2, 0, fake, 12, 0, 0, 0.0, 0, None) == hap.HAP_E_ARG
    assert lib.hap_build_similarity(fake, 10, 2, 1, 0, fake, 12, 0, 0, 0.0, 0, None) == hap.HAP_E_ARG
    # noise is defined for FP64 output only
    assert lib.hap_build_similarity(fake, 10, 2, 2, 0, fake, 12, 0, 0, 1e-12, 0, None) == hap.HAP_E_DTYPE
    d = ctypes.c_double()
    assert lib.hap_median_offdiag(fake, 1, 4, 0, ctypes.byref(d), None) == hap.HAP_E_ARG
    assert lib.hap_median_offdiag(fake, 10, 10, 0, ctypes.byref(d), None) == hap.HAP_E_ARG


def test_mlp_sizes_and_argument_checks(lib):
    # W1 32x128, b1, W2 128x128, b2, W3 128x3, b3
    assert lib.hap_mlp_param_count(32, 128, 3) == 32 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3
    assert lib.hap_mlp_param_count(0, 128, 3) == -1
    b = ctypes.c_size_t()
    assert lib.hap_mlp_workspace_size(32, 128, 3, 4096, ctypes.byref(b)) == hap.HAP_OK
    assert b.value >= 4 * 4096 * 128 * 4           # two activations and two deltas of 4096 x 128
    assert lib.hap_mlp_workspace_size(32, 128, 3, -1, ctypes.byref(b)) == hap.HAP_E_ARG
    fake = ctypes.c_void_p(4096)  # never dereferenced: every call below fails its checks first
    big = 1 << 40
    assert lib.hap_mlp_forward(None, 32, 128, 3, hap.HAP_F32, fake, 32, 10, fake, 3, fake, big, None) == hap.HAP_E_ARG
    assert lib.hap_mlp_forward(fake, 32, 128, 3, hap.HAP_F64, fake, 32, 10, fake, 3, fake, big, None) == hap.HAP_E_DTYPE
    assert lib.hap_mlp_forward(fake, 32, 128, 3, hap.HAP_F32, fake, 31, 10, fake, 3, fake, big, None) == hap.HAP_E_ARG
    assert lib.hap_mlp_forward(fake, 32, 128, 3, hap.HAP_F32, fake, 32, 10, fake, 3, fake, 16, None) == hap.HAP_E_ARG
    assert lib.hap_mlp_adam(fake, fake, fake, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == hap.HAP_E_ARG
    assert lib.hap_mlp_adam(fake, fake, fake, 10, 1, 1e-3, 1.0, 0.999, 1e-8, None) == hap.HAP_E_ARG
    assert lib.hap_mlp_train(fake, fake, 32, 128, 3, hap.HAP_BF16, 0, fake, 32, fake, 3, 100, fake, 0, 5, 1e-3,
                             None, fake, big, None) == hap.HAP_E_ARG


def test_warm_calls_reject_a_null_context(lib):
    fake = ctypes.c_void_p(4096)
    assert lib.hap_warm_features(None, fake, 32) == hap.HAP_E_ARG
    assert lib.hap_warm_targets(None, fake, 3) == hap.HAP_E_ARG
    assert lib.hap_set_warm_start(None, None, 0) == hap.HAP_E_ARG
    assert lib.hap_set_warm_alpha(None, fake, 3) == hap.HAP_E_ARG
    assert lib.hap_iterate_warm(None, None, 0, 10, 5, None, None, None) == hap.HAP_E_ARG
    assert lib.hap_iterate_warm_judged(None, fake, 1, 10, 5, None, 0, 0, 0, None, None, None, None,
                                       None) == hap.HAP_E_ARG


def test_batch_planning_checks_arguments(lib):
    b = ctypes.c_size_t()
    sizes = (ctypes.c_int32 * 3)(100, 2048, 2)
    assert lib.hap_batch_workspace_size(3, sizes, 16, 3, ctypes.byref(b)) == hap.HAP_OK
    # per problem: S, then R and A per level (n x ld floats each), plus vectors
    need = sum(n * ((n + 63) // 64 * 64) * 4 * (1 + 2 * 3) for n in (100, 2048, 2))
    assert need <= b.value < need * 1.1
    assert lib.hap_batch_workspace_size(3, sizes, 16, 3, None) == hap.HAP_E_ARG
    assert lib.hap_batch_workspace_size(0, sizes, 16, 3, ctypes.byref(b)) == hap.HAP_E_ARG
    assert lib.hap_batch_workspace_size(3, None, 16, 3, ctypes.byref(b)) == hap.HAP_E_ARG
    assert lib.hap_batch_workspace_size(3, sizes, 33, 3, ctypes.byref(b)) == hap.HAP_E_ARG
    assert lib.hap_batch_workspace_size(3, sizes, 16, 0, ctypes.byref(b)) == hap.HAP_E_ARG
    for bad in (1, 2049):
        one = (ctypes.c_int32 * 1)(bad)
        assert lib.hap_batch_workspace_size(1, one, 16, 3, ctypes.byref(b)) == hap.HAP_E_ARG
        assert b"2048" in lib.hap_last_error()
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(4096 + 1)     # misaligned: rejected before any device call
    assert lib.hap_batch_create(ctypes.byref(out), 3, sizes, 16, 3, fake, 1 << 40, None) == hap.HAP_E_ARG
    assert lib.hap_batch_create(None, 3, sizes, 16, 3, None, 0, None) == hap.HAP_E_ARG
    assert not out.value
    assert lib.hap_batch_set_launch(None, 512, 1, 4) == hap.HAP_E_ARG
    assert lib.hap_batch_destroy(None) == hap.HAP_OK


def test_bandwidth_probe_checks_arguments(lib):
    fake = (ctypes.c_void_p * 3)(4096, 8192, 12288)     # never dereferenced: every call fails its checks
    outs = (ctypes.c_void_p * 2)(16384, 20480)
    assert lib.hap_bandwidth_probe(2, 1, fake, outs, 64, 64, 64, 32, 0, None) == hap.HAP_E_ARG     # mix
    assert lib.hap_bandwidth_probe(1, 1, fake, outs, 64, 63, 64, 32, 0, None) == hap.HAP_E_ARG     # cols % 4
    assert lib.hap_bandwidth_probe(1, 1, fake, outs, 64, 64, 60, 32, 0, None) == hap.HAP_E_ARG     # ld < cols
    assert lib.hap_bandwidth_probe(1, 1, fake, outs, 64, 8196, 8196, 32, 0, None) == hap.HAP_E_UNSUPPORTED
    assert lib.hap_bandwidth_probe(1, 0, fake, None, 64, 64, 64, 32, 0, None) == hap.HAP_E_ARG     # no sink
    assert lib.hap_bandwidth_probe(0, 1, None, None, 64, 64, 64, 32, 0, None) == hap.HAP_E_ARG     # no output
    assert lib.hap_bandwidth_probe(0, 2, None, outs, 64, 64, 64, 32, 0, None) == hap.HAP_E_ARG     # mix
    assert lib.hap_bandwidth_probe(1, 1, fake, outs, 64, 64, 64, 32, 4, None) == hap.HAP_E_ARG     # flags
    import torch
    a = torch.zeros((8, 8))
    with pytest.raises(ValueError):
        hap.bandwidth_probe([a], [])                       # host tensors, no sink: refused before the call
    with pytest.raises(ValueError):
        hap.bandwidth_probe([a], [torch.zeros((8, 4))])    # shapes differ
