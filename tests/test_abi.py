"""The C-ABI library loads and exports every entry point its header declares (CPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "simpgmg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sgmg_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2604_26441_amd import simpgmg
    lib = ctypes.CDLL(simpgmg.library_path())
    names = _declared()
    assert "sgmg_pcg_solve" in names and "sgmg_vcycle" in names
    for n in names:
        getattr(lib, n)                    # raises AttributeError if missing
    assert set(names) == set(simpgmg.EXPORTS)


def test_default_options_match_paper_defaults():
    from paper_2604_26441_amd import simpgmg
    o = simpgmg.default_options(16, 8, 8)
    assert (o.nx, o.ny, o.nz) == (16, 8, 8)
    assert o.nu == 0.3 and o.Emin == 1e-9 and o.penal == 3.0
    assert o.n_levels == 4 and o.fine_degree == 2 and o.coarse_sweeps == 2
    assert abs(o.cheb_alpha - 1 / 30) < 1e-16 and o.jacobi_omega_max == 0.5
    assert o.power_iters_fine == 20 and o.power_iters_coarse == 10
    assert o.dense_max == 5000 and o.coarse_pcg_iters == 80


def test_struct_layout_matches_header(tmp_path):
    from paper_2604_26441_amd import simpgmg
    c = tmp_path / "sz.c"
    c.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "%s"\n'
                 'int main(){printf("%%zu %%zu %%zu %%zu\\n", sizeof(sgmg_options),'
                 ' offsetof(sgmg_options, seed), offsetof(sgmg_options, use_graphs),'
                 ' sizeof(sgmg_solve_info)); return 0;}\n' % HEADER)
    exe = tmp_path / "sz"
    r = subprocess.run(["gcc", str(c), "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("no host C compiler: " + r.stderr[:200])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals == [ctypes.sizeof(simpgmg.Options), simpgmg.Options.seed.offset,
                    simpgmg.Options.use_graphs.offset, ctypes.sizeof(simpgmg.SolveInfo)]


def test_setup_rejects_uncoarsenable_meshes_before_device_work():
    """A mesh with an axis of one element has no coarse level: setup must
    return SGMG_EINVAL from argument checking alone (no allocation, no
    kernel), also when the depth is automatic (n_levels = 0).  The element
    array pointer is never dereferenced on this path."""
    from paper_2604_26441_amd import simpgmg
    lib = ctypes.CDLL(simpgmg.library_path())
    lib.sgmg_setup_hierarchy.restype = ctypes.c_int
    lib.sgmg_last_error.restype = ctypes.c_char_p
    for dims, L in [((1, 4, 4), 0), ((4, 1, 4), 0), ((4, 4, 1), 2), ((1, 1, 1), 4)]:
        o = simpgmg.default_options(*dims, n_levels=L)
        h = ctypes.c_void_p()
        rc = lib.sgmg_setup_hierarchy(ctypes.byref(o), ctypes.c_void_p(64), None, None,
                                      ctypes.byref(h))
        assert rc == -1 and not h.value
        assert b"dims" in lib.sgmg_last_error()


def test_batch_item_layout_fits_its_allocation():
    """The per-item work memory of the batched solve (the layout whose
    256-byte rounding once overran its allocation) for every system of the
    32-system batch workload at 4 levels, and for 2..8 level hierarchies of
    odd meshes: sub-buffers are 256-byte aligned, each holds its vector,
    none overlaps the next, and the last one ends inside the allocation."""
    from paper_2604_26441_amd import simpgmg
    import workloads

    def levels(dims, L):
        out = [dims]
        for _ in range(L - 1):
            out.append(tuple(d // 2 for d in out[-1]))
        return out

    cases = [(d, 4) for d in workloads.batch_config()[0]]
    cases += [((17, 9, 5), 2), ((33, 17, 9), 3), ((255, 129, 129), 8), ((48, 24, 24), 5)]
    for dims, L in cases:
        lv = levels(dims, L)
        assert min(lv[-1]) >= 1
        ndofs = [3 * (a + 1) * (b + 1) * (c + 1) for a, b, c in lv]
        nxL, nyL, nzL = lv[-1]
        n_free = 3 * nxL * (nyL + 1) * (nzL + 1)
        total, bufs = simpgmg.batch_item_layout(ndofs, n_free)
        need = [8 * ndofs[0]] * 5 + [4 * ndofs[0]] * 5
        for l in range(1, L):
            need += [8 * ndofs[l]] * 4
        need.append(8 * max(n_free, 1))
        assert [s for _, s in bufs] == need
        for k, (off, size) in enumerate(bufs):
            assert off % 256 == 0
            end = off + size
            nxt = bufs[k + 1][0] if k + 1 < len(bufs) else total
            assert end <= nxt
        assert bufs[-1][0] + bufs[-1][1] <= total < bufs[-1][0] + bufs[-1][1] + 256
    import pytest
    with pytest.raises(simpgmg.SimpGmgError):
        simpgmg.batch_item_layout([100], 10)


def test_one_launch_batch_solve_checks_arguments_before_device_work():
    """sgmg_pcg_solve_batch_graph rejects a missing batch and a step count
    that is odd, below 2 or above 1024 with SGMG_EINVAL from its argument
    checks alone: the batch pointer (here a dummy) is not dereferenced."""
    from paper_2604_26441_amd import simpgmg
    lib = ctypes.CDLL(simpgmg.library_path())
    fn = lib.sgmg_pcg_solve_batch_graph
    fn.restype = ctypes.c_int
    vp = ctypes.c_void_p
    fn.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(vp),
                   ctypes.POINTER(vp), ctypes.c_double, ctypes.c_int, ctypes.c_int, vp,
                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), vp]
    lib.sgmg_last_error.restype = ctypes.c_char_p
    sysarr = (ctypes.c_int * 1)(0)
    fa = (vp * 1)(64)
    ua = (vp * 1)(128)
    nl, ms = ctypes.c_int(-7), ctypes.c_double(-1.0)
    cases = [(None, 2), (vp(64), 0), (vp(64), 3), (vp(64), 1026), (vp(64), -2)]
    for b, steps in cases:
        rc = fn(b, 1, sysarr, fa, ua, 1e-6, 10, steps, None, ctypes.byref(nl), ctypes.byref(ms),
                None)
        assert rc == -1, (b, steps)
        assert b"bad batch solve arguments" in lib.sgmg_last_error()
    assert nl.value == -7 and ms.value == -1.0       # outputs untouched on rejection
