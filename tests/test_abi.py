"""The C-ABI library loads, exports every symbol the header declares, and
rejects bad arguments on the host before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlgl.h")
LIB = os.path.join(ROOT, "paper_2008_02710_amd", "librlgl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rlgl_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2008_02710_amd.build as b
        b.build(force=True)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "rlgl_create" in names and "rlgl_solve" in names and "rlgl_step" in names and "rlgl_destroy" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    import paper_2008_02710_amd as rl
    for name in declared_functions():
        assert hasattr(rl, name), name


def test_struct_sizes_match_header(tmp_path):
    """The ctypes mirrors have the C layout (checked against offsets the
    compiler computes for the header)."""
    import paper_2008_02710_amd as rl
    src = str(tmp_path / "sizes_probe.c")
    exe = str(tmp_path / "sizes_probe")
    open(src, "w").write(
        '#include <stdio.h>\n#include <stddef.h>\n#include "rlgl.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(rlgl_graph),'
        ' sizeof(rlgl_options), sizeof(rlgl_step_info), sizeof(rlgl_kernel_stat),'
        ' offsetof(rlgl_options, record_green), offsetof(rlgl_step_info, last_route),'
        ' sizeof(rlgl_batch_graphs), sizeof(rlgl_batch_options), offsetof(rlgl_batch_options, check_period),'
        ' sizeof(rlgl_chain_result), sizeof(rlgl_pool_options), sizeof(rlgl_request),'
        ' offsetof(rlgl_request, tol_l1), offsetof(rlgl_options, relabel), offsetof(rlgl_options, seed),'
        ' offsetof(rlgl_batch_options, relabel));'
        'return 0;}\n')
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, src])
    out = subprocess.check_output([exe]).decode().split()
    got = [ctypes.sizeof(rl.rlgl_graph), ctypes.sizeof(rl.rlgl_options), ctypes.sizeof(rl.rlgl_step_info),
           ctypes.sizeof(rl.rlgl_kernel_stat), rl.rlgl_options.record_green.offset,
           rl.rlgl_step_info.last_route.offset, ctypes.sizeof(rl.rlgl_batch_graphs),
           ctypes.sizeof(rl.rlgl_batch_options), rl.rlgl_batch_options.check_period.offset,
           ctypes.sizeof(rl.rlgl_chain_result), ctypes.sizeof(rl.rlgl_pool_options), ctypes.sizeof(rl.rlgl_request),
           rl.rlgl_request.tol_l1.offset, rl.rlgl_options.relabel.offset, rl.rlgl_options.seed.offset,
           rl.rlgl_batch_options.relabel.offset]
    assert [int(x) for x in out] == got


def test_host_side_argument_checks():
    import paper_2008_02710_amd as rl
    g = rl.rlgl_graph(10, 0, 1, 0, None, None, None, None, 0.85)
    opt = rl.rlgl_default_options()
    assert opt.sched == rl.SCHED_THRESHOLD and opt.r == 1.0 and opt.theta_period == 1
    assert rl.rlgl_workspace_bytes(g, opt) > 0
    bad = rl.rlgl_graph(0, 0, 1, 0, None, None, None, None, 0.85)
    assert rl.rlgl_workspace_bytes(bad, opt) == 0
    ctx = ctypes.c_void_p()
    lib = rl._lib
    # damping outside (0, 1]
    g0 = rl.rlgl_graph(10, 0, 1, 0, None, None, None, None, 0.0)
    assert lib.rlgl_create(ctypes.byref(g0), ctypes.byref(opt), 4096, 1 << 20, None, ctypes.byref(ctx)) == rl.RLGL_EINVAL
    assert "damping" in rl.rlgl_last_error()
    # workspace too small
    assert lib.rlgl_create(ctypes.byref(g), ctypes.byref(opt), 4096, 16, None, ctypes.byref(ctx)) == rl.RLGL_ENOMEM
    # bad options
    for field, value in (("sched", 9), ("r", 0.5), ("theta_period", 0), ("precision", 7), ("route", 5)):
        o = rl.rlgl_default_options(**{field: value})
        assert lib.rlgl_create(ctypes.byref(g), ctypes.byref(o), 4096, 1 << 30, None, ctypes.byref(ctx)) == rl.RLGL_EINVAL
    for sched in (rl.SCHED_TOPK, rl.SCHED_PC):
        o = rl.rlgl_default_options(sched=sched, k=5, relabel=1)
        assert lib.rlgl_create(ctypes.byref(g), ctypes.byref(o), 4096, 1 << 30, None,
                               ctypes.byref(ctx)) == rl.RLGL_EINVAL
        assert "relabel" in rl.rlgl_last_error()
    # the relabelled layout needs room for a second copy of the graph
    o = rl.rlgl_default_options(relabel=1)
    g2 = rl.rlgl_graph(1000, 5000, 1, 1, None, 1, 1, None, 0.85)
    assert rl.rlgl_workspace_bytes(g2, o) >= rl.rlgl_workspace_bytes(g2, rl.rlgl_default_options()) + 8 * 5000
    o = rl.rlgl_default_options(sched=rl.SCHED_TOPK, k=0)
    assert lib.rlgl_create(ctypes.byref(g), ctypes.byref(o), 4096, 1 << 30, None, ctypes.byref(ctx)) == rl.RLGL_EINVAL
    # pull routing without the CSC
    o = rl.rlgl_default_options(route=rl.ROUTE_PULL)
    assert lib.rlgl_create(ctypes.byref(g), ctypes.byref(o), 4096, 1 << 30, None, ctypes.byref(ctx)) == rl.RLGL_EINVAL
    assert ctx.value is None


def test_pool_host_side_checks():
    import paper_2008_02710_amd as rl
    lib = rl._lib
    o = rl.rlgl_pool_default_options()
    assert o.sched == rl.SCHED_THRESHOLD and o.precision == rl.FP32C_KAHANH and o.max_chains == 256
    ws = rl.rlgl_pool_workspace_bytes(o, 1 << 30)
    assert ws >= 1 << 30
    # footprints grow with the chain and bound its arrays
    f1, f2 = rl.rlgl_pool_footprint(o, 1000, 10000), rl.rlgl_pool_footprint(o, 100000, 1000000)
    assert 0 < f1 < f2 and f2 >= 4 * 1000000 + 32 * 100000
    assert rl.rlgl_pool_footprint(o, 0, 0) == 0
    for field, value in (("sched", rl.SCHED_TOPK), ("r", 0.5), ("precision", 5), ("wg_size", 128),
                         ("max_chains", 0), ("max_steps", -1)):
        bad = rl.rlgl_pool_default_options(**{field: value})
        assert rl.rlgl_pool_workspace_bytes(bad, 1 << 20) == 0, field
        h = ctypes.c_void_p()
        assert lib.rlgl_pool_create(ctypes.byref(bad), 4096, 1 << 30, None, ctypes.byref(h)) == rl.RLGL_EINVAL
    h = ctypes.c_void_p()
    assert lib.rlgl_pool_create(ctypes.byref(o), None, 1 << 30, None, ctypes.byref(h)) == rl.RLGL_EINVAL
    assert lib.rlgl_pool_create(ctypes.byref(o), 4096, 1024, None, ctypes.byref(h)) == rl.RLGL_ENOMEM
    assert h.value is None
    slot = ctypes.c_int32(-1)
    req = rl.rlgl_request(10, 0, None, None, None, 0.85, 1e-6)
    assert lib.rlgl_pool_admit(None, ctypes.byref(req), ctypes.byref(slot)) == rl.RLGL_EINVAL
    assert lib.rlgl_pool_poll(None, None, 0) == rl.RLGL_EINVAL
    assert lib.rlgl_pool_release(None, 0) == rl.RLGL_EINVAL


def test_small_solver_host_side_checks():
    """rlgl_solve_small rejects bad arguments before any launch; its workspace
    size follows n (history and moved cash, 8 bytes each per node)."""
    import paper_2008_02710_amd as rl
    lib = rl._lib
    assert rl.rlgl_small_workspace_bytes(0) == 0
    w1, w2 = rl.rlgl_small_workspace_bytes(1000), rl.rlgl_small_workspace_bytes(2000)
    assert w2 - w1 >= 2 * (8 * 1000 - 256) and w1 >= 16 * 1000
    assert rl.rlgl_small_max_n(9) == 0
    g = rl.rlgl_graph(10, 0, 1, 0, None, 1, 0, None, 0.85)
    info = rl.rlgl_step_info()
    for field, value in (("sched", rl.SCHED_TOPK), ("r", 0.5), ("theta_period", 0), ("precision", 7)):
        o = rl.rlgl_default_options(**{field: value})
        assert lib.rlgl_solve_small(ctypes.byref(g), ctypes.byref(o), 1e-9, 10, None, 4096, 1 << 20, None,
                                    ctypes.byref(info)) == rl.RLGL_EINVAL
    o = rl.rlgl_default_options(sched=rl.SCHED_MAXC)
    nocsc = rl.rlgl_graph(10, 0, 1, 0, None, None, None, None, 0.85)
    assert lib.rlgl_solve_small(ctypes.byref(nocsc), ctypes.byref(o), 1e-9, 10, None, 4096, 1 << 20, None,
                                ctypes.byref(info)) == rl.RLGL_EINVAL
    assert "CSC" in rl.rlgl_last_error()
    g0 = rl.rlgl_graph(10, 0, 1, 0, None, 1, 0, None, 1.5)
    assert lib.rlgl_solve_small(ctypes.byref(g0), ctypes.byref(o), 1e-9, 10, None, 4096, 1 << 20, None,
                                ctypes.byref(info)) == rl.RLGL_EINVAL
    assert lib.rlgl_solve_small(ctypes.byref(g), ctypes.byref(o), -1.0, 10, None, 4096, 1 << 20, None,
                                ctypes.byref(info)) == rl.RLGL_EINVAL


def test_static_workspace_size_matches_header():
    import paper_2008_02710_amd as rl
    text = open(HEADER).read()
    m = re.search(r"#define\s+RLGL_SMALL_STATIC_BYTES\s+\((\d+)u\s*\*\s*(\d+)u\)", text)
    assert m, "RLGL_SMALL_STATIC_BYTES not found"
    assert int(m.group(1)) * int(m.group(2)) == rl.RLGL_SMALL_STATIC_BYTES
    # the largest one-workgroup workspace the static array holds
    assert rl.rlgl_small_workspace_bytes(32736) <= rl.RLGL_SMALL_STATIC_BYTES
    assert rl.rlgl_small_workspace_bytes(32737) > rl.RLGL_SMALL_STATIC_BYTES
    g = rl.rlgl_graph(40000, 0, 1, 0, None, 1, 0, None, 0.85)
    o = rl.rlgl_default_options(precision=rl.FP32C_FP64H)
    info = rl.rlgl_step_info()
    assert rl._lib.rlgl_solve_small_static(ctypes.byref(g), ctypes.byref(o), 1e-9, 10, None, None,
                                           ctypes.byref(info)) == rl.RLGL_EINVAL
    assert "static" in rl.rlgl_last_error()
