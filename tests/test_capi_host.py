"""The C ABI on the host (CPU only): the library loads, exports every function
include/resample.h declares, and rejects bad arguments before any launch.
No kernel is enqueued by these tests."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1202_6163_amd", "libresample.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libresample.so not built")


@pytest.fixture(scope="module")
def L():
    from paper_1202_6163_amd import _lib
    return _lib


def test_exports_every_declared_function(L):
    names = L.header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L.lib, name), name
    # and the shared object's dynamic symbol table agrees
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    assert set(names) <= exported


def test_strerror_and_version(L):
    assert L.lib.rs_strerror(0) == b"success"
    assert L.lib.rs_strerror(-1) == b"invalid argument"
    assert L.lib.rs_strerror(-2) == b"workspace too small"
    assert L.lib.rs_strerror(12345) == b"unknown error"
    assert L.lib.rs_version() >= 100


def test_argument_errors_before_launch(L):
    lib = L.lib
    fake = ctypes.c_void_p(0x10000000)
    other = ctypes.c_void_p(0x20000000)
    ws = ctypes.c_void_p(0x30000000)
    # null pointers, negative sizes, P beyond int32 ancestors
    assert lib.resample_metropolis(None, other, 10, 4, 1, 0, None, None) == L.RS_EINVAL
    assert lib.resample_metropolis(fake, other, -1, 4, 1, 0, None, None) == L.RS_EINVAL
    assert lib.resample_metropolis(fake, other, 2**31, 4, 1, 0, None, None) == L.RS_EINVAL
    # overlapping input and output
    assert lib.resample_metropolis(fake, ctypes.c_void_p(0x10000004), 10, 4, 1, 0, None,
                                   None) == L.RS_EINVAL
    third = ctypes.c_void_p(0x40000000)
    for fn in (lib.resample_stratified, lib.resample_systematic, lib.resample_multinomial):
        if fn is lib.resample_multinomial:
            call = fn
        else:  # stratified/systematic take an offspring pointer after anc
            def call(lw, anc, *rest, fn=fn):
                return fn(lw, anc, None, *rest)
        assert call(None, other, 10, 1, 0, None, ws, 1 << 20, None, None) == L.RS_EINVAL
        assert call(fake, other, 10, 1, 0, None, None, 1 << 20, None, None) == L.RS_EINVAL
        assert call(fake, other, 10, 1, 0, None, ws, 1, None, None) == L.RS_EWORKSPACE
        assert call(fake, fake, 10, 1, 0, None, ws, 1 << 20, None, None) == L.RS_EINVAL
        assert call(fake, None, 10, 1, 0, None, ws, 1 << 20, None, None) == L.RS_EINVAL
    for fn in (lib.resample_stratified, lib.resample_systematic):
        # offspring only is valid up to the launch; overlapping outputs are not
        assert fn(fake, None, third, 10, 1, 0, None, ws, 1, None, None) == L.RS_EWORKSPACE
        assert fn(fake, other, ctypes.c_void_p(0x20000008), 10, 1, 0, None, ws, 1 << 20, None,
                  None) == L.RS_EINVAL
        assert fn(fake, other, third, 10, 1, 0, ctypes.c_void_p(0x40000010), ws, 1 << 20, None,
                  None) == L.RS_EINVAL
        assert fn(fake, other, ctypes.c_void_p(0x30000000), 10, 1, 0, None, ws, 1 << 20, None,
                  None) == L.RS_EINVAL
    assert lib.permute_copy(fake, other, other, 10, 4, None, None) == L.RS_EINVAL
    assert lib.permute_copy(fake, other, ws, 10, 0, None, None) == L.RS_EINVAL
    assert lib.ancestors_to_offspring(fake, fake, 10, None, None) == L.RS_EINVAL
    assert lib.rs_log_sum_exp(fake, 10, other, ws, 1, None, None) == L.RS_EWORKSPACE
    assert lib.rs_log_u_table(None, None, None) == L.RS_EINVAL


def test_empty_resampling_is_a_no_op(L):
    lib = L.lib
    assert lib.resample_metropolis(None, None, 0, 4, 1, 0, None, None) == L.RS_OK
    assert lib.resample_stratified(None, None, None, 0, 1, 0, None, None, 0, None, None) == L.RS_OK
    assert lib.permute_copy(None, None, None, 0, 4, None, None) == L.RS_OK
    assert lib.ancestors_to_offspring(None, None, 0, None, None) == L.RS_OK


def test_workspace_bytes(L):
    lib = L.lib
    assert lib.rs_workspace_bytes(0, 0) == 0
    assert lib.rs_workspace_bytes(1 << 20, L.METROPOLIS) == 0
    prev = 0
    for P in (1, 1000, 1024, 1025, 1 << 20, (1 << 31) - 1):
        b = lib.rs_workspace_bytes(P, L.STRATIFIED)
        assert b >= prev and b % 256 == 0
        prev = b
        assert lib.rs_workspace_bytes(P, L.MULTINOMIAL) >= b + 8 * P
        assert lib.rs_workspace_bytes(P, L.SYSTEMATIC) == b


def test_tuning_validation(L):
    t = L.Tuning()
    assert L.lib.rs_metropolis_get_tuning(ctypes.byref(t)) == 0
    saved = L.Tuning(t.block, t.unroll, t.lds_max_p, t.lanes_per_chain)
    for bad in ((32, 8, 0, 0), (256, 3, 0, 0), (256, 8, -1, 0), (256, 8, 0, 3), (2048, 8, 0, 0)):
        assert L.lib.rs_metropolis_set_tuning(ctypes.byref(L.Tuning(*bad))) == L.RS_EINVAL
    assert L.lib.rs_metropolis_set_tuning(ctypes.byref(L.Tuning(512, 4, 1000, 8))) == 0
    assert L.lib.rs_metropolis_get_tuning(ctypes.byref(t)) == 0
    assert (t.block, t.unroll, t.lds_max_p, t.lanes_per_chain) == (512, 4, 1000, 8)
    assert L.lib.rs_metropolis_set_tuning(ctypes.byref(saved)) == 0


def test_metropolis_B_matches_oracle(L):
    rng = np.random.default_rng(11)
    for _ in range(2000):
        P = int(rng.integers(1, 1 << 24))
        w_max = float(np.exp(rng.uniform(np.log(1.0 / P), 0)))
        eps = float(10 ** rng.uniform(-4, -0.5))
        assert L.lib.metropolis_B(P, w_max, eps) == oracle.metropolis_B(P, w_max, eps)
    assert L.lib.metropolis_B(4096, 1.0 / 4096, 1e-3) == 1
    assert L.lib.metropolis_B(1, 1.0, 1e-3) == 0
    assert L.lib.metropolis_B(100, 0.0, 1e-3) == 0


def test_struct_layouts_match_header(L, tmp_path):
    # the ctypes mirrors must have the C layout of include/resample.h
    import subprocess
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "resample.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(rs_instance), '
        'offsetof(rs_instance, P), offsetof(rs_instance, seed), sizeof(rs_batch_tuning), '
        'sizeof(rs_batch_plan), offsetof(rs_batch_plan, smem_main), '
        'sizeof(rs_metropolis_tuning));return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(L.Instance), L.Instance.P.offset, L.Instance.seed.offset,
            ctypes.sizeof(L.BatchTuning), ctypes.sizeof(L.BatchPlan), L.BatchPlan.smem_main.offset,
            ctypes.sizeof(L.Tuning)]
    assert got == want


def test_batch_plan_validation_before_any_upload(L):
    lib = L.lib

    def inst(kind, P=100, lw=0x1000000, anc=0x2000000, off=None, x_in=None, x_out=None, D=0, B=8):
        return L.Instance(lw=lw, anc=anc, off=off, x_in=x_in, x_out=x_out, status=None, P=P, D=D,
                          kind=kind, B=B, instance=0, seed=1)

    def plan_bytes(*insts):
        return lib.rs_batch_plan_bytes((L.Instance * len(insts))(*insts), len(insts), None)

    good = inst(L.METROPOLIS)
    arr = (L.Instance * 1)(good)
    assert lib.rs_batch_plan_bytes(arr, 1, None) > 0
    assert lib.rs_batch_workspace_bytes(arr, 1) == 0
    assert plan_bytes(inst(77)) == 0                                      # unknown kind
    assert plan_bytes(inst(L.METROPOLIS, anc=0x1000010)) == 0             # lw/anc overlap
    assert plan_bytes(inst(L.STRATIFIED, x_in=0x3000000, D=4)) == 0       # copy without x_out
    assert plan_bytes(inst(L.METROPOLIS, anc=None)) == 0                  # Metropolis needs anc
    assert plan_bytes(inst(L.METROPOLIS, off=0x4000000)) == 0             # and has no offspring
    assert plan_bytes(inst(L.STRATIFIED, anc=None)) == 0                  # no output at all
    assert plan_bytes(inst(L.STRATIFIED, anc=None, off=0x4000000)) > 0    # offspring only
    assert plan_bytes(inst(L.SYSTEMATIC, off=0x2000100)) == 0             # anc/off overlap
    bad_tuning = L.BatchTuning(300, 8, 0, 0)
    assert lib.rs_batch_plan_bytes(arr, 1, ctypes.byref(bad_tuning)) == 0
    plan = L.BatchPlan()
    # plan buffer too small / missing workspace: rejected before the upload
    assert lib.rs_batch_plan_init(ctypes.byref(plan), arr, 1, None, ctypes.c_void_p(0x4000000), 1,
                                  None, 0, None, None) == L.RS_EWORKSPACE
    strat = (L.Instance * 1)(inst(L.STRATIFIED, P=5000, B=0))
    need = lib.rs_batch_plan_bytes(strat, 1, None)
    assert lib.rs_batch_workspace_bytes(strat, 1) >= lib.rs_workspace_bytes(5000, L.STRATIFIED)
    assert lib.rs_batch_plan_init(ctypes.byref(plan), strat, 1, None, ctypes.c_void_p(0x4000000),
                                  need, None, 0, None, None) == L.RS_EWORKSPACE
    assert lib.resample_batch(None, None) == L.RS_EINVAL


def test_filter_argument_errors(L):
    lib = L.lib
    f = ctypes.c_void_p
    assert lib.filter_init(None, 10, 8, 1, None) == L.RS_EINVAL
    assert lib.filter_init(f(0x1000), 10, 65, 1, None) == L.RS_EINVAL
    assert lib.filter_loglik(None, 10, 8, f(0x1000), None) == L.RS_EINVAL
    assert lib.filter_loglik(f(0x1000), -1, 8, f(0x9000), None) == L.RS_EINVAL
    assert lib.filter_loglik(f(0x1000), 10, 0, f(0x9000), None) == L.RS_EINVAL
    assert lib.filter_loglik(f(0x1000), 10, 8, f(0x1008), None) == L.RS_EINVAL  # out inside lse
    assert lib.filter_propagate_weight(f(0x1000), f(0x1000), f(0x90000), 10, 4, f(0x80000),
                                       f(0x70000), 0.1, 0.5, 1, 1, None) == L.RS_EINVAL
    assert lib.filter_propagate_weight(f(0x1000), f(0x20000), f(0x90000), 10, 4, f(0x80000),
                                       f(0x70000), 0.1, 0.0, 1, 1, None) == L.RS_EINVAL
    assert lib.resample_metropolis_adaptive(f(0x1000), f(0x20000), 10, 0.0, 64, 1, 0,
                                            f(0x90000), 1 << 20, None, None, None) == L.RS_EINVAL
    assert lib.resample_metropolis_adaptive(f(0x1000), f(0x20000), 10, 0.01, 64, 1, 0,
                                            f(0x90000), 8, None, None, None) == L.RS_EWORKSPACE


def test_probe_argument_errors(L):
    lib = L.lib
    f = ctypes.c_void_p
    assert lib.rs_probe_gather(None, 10, 256, 1, 1, f(0x1000), None) == L.RS_EINVAL
    assert lib.rs_probe_gather(f(0x1000), 10, 100, 1, 1, f(0x8000), None) == L.RS_EINVAL
    assert lib.rs_probe_gather(f(0x1000), 0, 256, 1, 1, f(0x8000), None) == L.RS_EINVAL
    assert lib.rs_probe_philox(1, 256, 0, f(0x8000), None) == L.RS_EINVAL
    assert lib.rs_probe_philox(1, 256, 1, None, None) == L.RS_EINVAL


def test_workspace_must_be_256_byte_aligned(L):
    # a workspace off a 256-byte boundary is refused before any launch, by
    # every entry point that takes one (with a large enough size, so the
    # alignment is the only fault)
    lib = L.lib
    f = ctypes.c_void_p
    lw, anc, xi, xo, out = f(0x100000), f(0x200000), f(0x400000), f(0x800000), f(0xA00000)
    big = 1 << 30
    for bad in (f(0xC00008), f(0xC00080)):
        for fn in (lib.resample_stratified, lib.resample_systematic):
            assert fn(lw, anc, None, 10, 1, 0, None, bad, big, None, None) == L.RS_EINVAL
        assert lib.resample_multinomial(lw, anc, 10, 1, 0, None, bad, big, None,
                                        None) == L.RS_EINVAL
        for kind in (L.STRATIFIED, L.SYSTEMATIC, L.MULTINOMIAL):
            assert lib.resample_and_copy(kind, lw, anc, None, 10, 8, 1, 0, xi, xo, 4, bad, big,
                                         None, None) == L.RS_EINVAL
            assert lib.resample_sorted(kind, lw, anc, 10, 1, 0, bad, big, None,
                                       None) == L.RS_EINVAL
        assert lib.rs_log_sum_exp(lw, 10, out, bad, big, None, None) == L.RS_EINVAL
        assert lib.rs_workspace_log_sum_exp(bad, 10, out, None) == L.RS_EINVAL
        assert lib.resample_metropolis_adaptive(lw, anc, 10, 0.01, 64, 1, 0, bad, big, None,
                                                None, None) == L.RS_EINVAL
    # the same calls with an aligned workspace get past the check (to the size test)
    good = f(0xC00000)
    assert lib.resample_multinomial(lw, anc, 10, 1, 0, None, good, 8, None,
                                    None) == L.RS_EWORKSPACE
    assert lib.rs_log_sum_exp(lw, 10, out, good, 8, None, None) == L.RS_EWORKSPACE


def test_sorted_variant_arguments(L):
    lib = L.lib
    f = ctypes.c_void_p
    assert lib.rs_sorted_workspace_bytes(1000, 3) == 0  # Metropolis has no sorted variant
    for kind in (L.STRATIFIED, L.SYSTEMATIC, L.MULTINOMIAL):
        b = lib.rs_sorted_workspace_bytes(1 << 16, kind)
        assert b >= lib.rs_workspace_bytes(1 << 16, kind) + 20 * (1 << 16)
        assert lib.resample_sorted(kind, None, None, 0, 1, 0, None, 0, None, None) == L.RS_OK
        assert lib.resample_sorted(kind, None, f(0x1000), 10, 1, 0, f(0x9000), b, None,
                                   None) == L.RS_EINVAL
        assert lib.resample_sorted(kind, f(0x1000), f(0x2000), 10, 1, 0, f(0x90000), 16, None,
                                   None) == L.RS_EWORKSPACE
    assert lib.resample_sorted(9, f(0x1000), f(0x2000), 10, 1, 0, f(0x90000), 1 << 30, None,
                               None) == L.RS_EINVAL


def test_resample_and_copy_arguments(L):
    lib = L.lib
    f = ctypes.c_void_p
    lw, anc, off, xi, xo, ws = (f(0x100000), f(0x200000), f(0x300000), f(0x400000), f(0x800000),
                                f(0xC00000))
    ok = dict(kind=L.METROPOLIS)

    def call(kind=3, lw=lw, anc=anc, off=None, P=10, xi=xi, xo=xo, D=4, ws=ws, wsb=1 << 20):
        return lib.resample_and_copy(kind, lw, anc, off, P, 8, 1, 0, xi, xo, D, ws, wsb, None,
                                     None)
    assert ok and call(P=0, lw=None, anc=None, xi=None, xo=None) == L.RS_OK
    assert call(kind=9) == L.RS_EINVAL
    assert call(anc=None) == L.RS_EINVAL
    assert call(xi=None) == L.RS_EINVAL
    assert call(D=0) == L.RS_EINVAL
    assert call(off=off) == L.RS_EINVAL                      # Metropolis has no offspring
    assert call(kind=L.MULTINOMIAL, off=off) == L.RS_EINVAL  # nor multinomial
    assert call(xo=f(0x400010)) == L.RS_EINVAL               # x_out overlaps x_in
    assert call(xo=f(0x200004)) == L.RS_EINVAL               # x_out overlaps anc
    assert call(kind=L.STRATIFIED, ws=None) == L.RS_EINVAL
    assert call(kind=L.STRATIFIED, wsb=8) == L.RS_EWORKSPACE
    assert call(kind=L.SYSTEMATIC, off=f(0x200008)) == L.RS_EINVAL  # off overlaps anc


def test_batched_filter_and_batch_step_arguments(L):
    lib = L.lib
    f = ctypes.c_void_p
    x, xo, lw, A, y, q = (f(0x100000), f(0x900000), f(0x1100000), f(0x1200000), f(0x1300000),
                          f(0x1400000))
    assert lib.filter_init_batch(None, 0, 10, 4, 1, None) == L.RS_OK      # K = 0: nothing to do
    assert lib.filter_init_batch(None, 2, 10, 4, 1, None) == L.RS_EINVAL
    assert lib.filter_init_batch(x, 2, 10, 65, 1, None) == L.RS_EINVAL    # D above 64
    assert lib.filter_init_batch(x, -1, 10, 4, 1, None) == L.RS_EINVAL
    ok = (x, xo, lw, 2, 10, 4, A, y, q, 0.5, 1, 1, None)
    args = list(ok)
    args[8] = None                                                      # q missing
    assert lib.filter_propagate_weight_batch(*args) == L.RS_EINVAL
    args = list(ok)
    args[9] = 0.0                                                       # r must be > 0
    assert lib.filter_propagate_weight_batch(*args) == L.RS_EINVAL
    args = list(ok)
    args[1] = f(0x100010)                                               # x_out overlaps x_in
    assert lib.filter_propagate_weight_batch(*args) == L.RS_EINVAL
    assert lib.resample_batch_at(None, 3, None) == L.RS_EINVAL
    assert lib.rs_batch_log_mean_weight(None, f(0x1000), None) == L.RS_EINVAL
    plan = L.BatchPlan()
    assert lib.rs_batch_log_mean_weight(ctypes.byref(plan), f(0x1000), None) == L.RS_EINVAL


def test_static_entry_arguments_and_limit(L):
    # the no-allocation entry point: the header's array size, every kind fits
    # P = 2^20, and bad arguments or sizes beyond the array are refused
    # before any launch (and before the array's address is looked up)
    hdr = open(os.path.join(ROOT, "include", "resample.h")).read()
    m = re.search(r"#define RS_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == L.RS_STATIC_SCRATCH_BYTES
    lib = L.lib
    for kind in (L.STRATIFIED, L.SYSTEMATIC, L.MULTINOMIAL):
        assert lib.rs_workspace_bytes(1 << 20, kind) <= L.RS_STATIC_SCRATCH_BYTES
    f = ctypes.c_void_p
    assert lib.resample_prefix_static(7, f(0x1000), f(0x90000), None, 10, 1, 0, None, None,
                                      None) == L.RS_EINVAL
    assert lib.resample_prefix_static(0, f(0x1000), f(0x90000), None, -1, 1, 0, None, None,
                                      None) == L.RS_EINVAL
    assert lib.resample_prefix_static(2, f(0x1000), f(0x90000000), None, 1 << 22, 1, 0, None,
                                      None, None) == L.RS_EWORKSPACE
    assert lib.resample_prefix_static(0, None, f(0x90000), None, 0, 1, 0, None, None,
                                      None) == L.RS_OK  # empty: nothing to do


def test_inplace_update_arguments(L):
    # the minimal-copy update: its workspace size, and every argument error
    # returned before a launch (the pointers are never dereferenced)
    lib = L.lib
    f = ctypes.c_void_p
    assert lib.rs_inplace_workspace_bytes(0) == 0
    sizes = [lib.rs_inplace_workspace_bytes(P) for P in (1, 1024, 1025, 1 << 20, 2**31 - 1)]
    assert all(a <= b for a, b in zip(sizes, sizes[1:])) and sizes[0] > 0
    P, D = 1000, 4
    off, x, anc = f(0x100000), f(0x200000), f(0x300000)
    ws, wsb = f(0x400000), lib.rs_inplace_workspace_bytes(P)
    call = lib.offspring_update_inplace
    assert call(None, None, 0, 0, None, None, 0, None, None) == L.RS_OK    # empty
    assert call(None, x, P, D, anc, ws, wsb, None, None) == L.RS_EINVAL    # no counts
    assert call(off, None, P, D, anc, ws, wsb, None, None) == L.RS_EINVAL  # no rows
    assert call(off, x, P, D, anc, None, wsb, None, None) == L.RS_EINVAL   # no workspace
    assert call(off, x, P, D, anc, f(0x400010), wsb, None, None) == L.RS_EINVAL  # misaligned
    assert call(off, x, P, 0, anc, ws, wsb, None, None) == L.RS_EINVAL     # D < 1
    assert call(off, x, -1, D, anc, ws, wsb, None, None) == L.RS_EINVAL
    assert call(off, x, 2**31, D, anc, ws, wsb, None, None) == L.RS_EINVAL
    assert call(off, f(0x100000 + 4 * P - 4), P, D, anc, ws, wsb, None, None) == L.RS_EINVAL
    assert call(off, x, P, D, f(0x200000 + 16), ws, wsb, None, None) == L.RS_EINVAL  # anc in x
    assert call(off, x, P, D, anc, ws, wsb - 1, None, None) == L.RS_EWORKSPACE
    assert call(off, x, P, D, anc, f(0x300000), wsb, None, None) == L.RS_EINVAL  # ws over anc
    # P * D beyond 2^40 state values is refused (no byte count overflows)
    assert call(off, x, 2**31 - 1, 2**30, None, ws, 1 << 62, None, None) == L.RS_EINVAL
    assert lib.permute_copy(off, x, f(0x900000000), 2**31 - 1, 2**30, None, None) == L.RS_EINVAL


def test_prefix_path_selection(L):
    # process-wide form of the stratified/systematic calls: unknown values are
    # refused and leave the setting unchanged
    lib = L.lib
    saved = lib.rs_prefix_get_path()
    try:
        for path in (L.PATH_LAUNCHES, L.PATH_ONEPASS, L.PATH_AUTO):
            assert lib.rs_prefix_set_path(path, -1) == L.RS_OK
            assert lib.rs_prefix_get_path() == path
        assert lib.rs_prefix_set_path(L.PATH_ONEPASS, 0) == L.RS_OK
        for bad in (-1, 3, 99):
            assert lib.rs_prefix_set_path(bad, -1) == L.RS_EINVAL
            assert lib.rs_prefix_get_path() == L.PATH_ONEPASS
    finally:
        lib.rs_prefix_set_path(saved, -1)


def test_offspring_ws_arguments(L):
    # the workspace form of ancestors_to_offspring: its size (0 beyond 2^24,
    # where it runs as the plain conversion) and argument errors before any launch
    lib = L.lib
    f = ctypes.c_void_p
    assert lib.rs_offspring_workspace_bytes(0) == 0
    assert lib.rs_offspring_workspace_bytes(1) > 0
    assert lib.rs_offspring_workspace_bytes(1 << 24) >= 4 << 24
    assert lib.rs_offspring_workspace_bytes((1 << 24) + 1) == 0
    P = 5000
    need = lib.rs_offspring_workspace_bytes(P)
    anc, off, ws = f(0x100000), f(0x200000), f(0x300000)
    call = lib.ancestors_to_offspring_ws
    assert call(None, None, 0, None, 0, None, None) == L.RS_OK           # empty
    assert call(None, off, P, ws, need, None, None) == L.RS_EINVAL
    assert call(anc, None, P, ws, need, None, None) == L.RS_EINVAL
    assert call(anc, off, -1, ws, need, None, None) == L.RS_EINVAL
    assert call(anc, off, 2**31, ws, need, None, None) == L.RS_EINVAL
    assert call(anc, f(0x100000 + 4 * P - 4), P, ws, need, None, None) == L.RS_EINVAL
    assert call(anc, off, P, None, need, None, None) == L.RS_EINVAL        # no workspace
    assert call(anc, off, P, f(0x300010), need, None, None) == L.RS_EINVAL  # misaligned
    assert call(anc, off, P, ws, need - 1, None, None) == L.RS_EWORKSPACE
    assert call(anc, off, P, f(0x200000), need, None, None) == L.RS_EINVAL  # ws over off
