"""Host-only checks of the boundary: the built library loads and exports every
entry point the headers declare, and the binding's structures match the C
layouts.  No device calls are made."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2408_08262_amd import airg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in ("airg.h", "airg_steps.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(airg_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(airg.LIB_PATH), "libairg.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", airg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    declared = declared_functions()
    assert declared, "no declarations parsed"
    missing = declared - exported
    assert not missing, "declared but not exported: %s" % sorted(missing)
    # and the binding knows every one of them
    assert declared <= set(airg.EXPORTS)


def test_library_loads_and_reports_defaults_without_a_device():
    L = airg.lib()
    for name in airg.EXPORTS:
        assert hasattr(L, name)
    o = airg.default_opts()
    assert o.struct_size == C.sizeof(airg.Opts)
    assert (o.strong_threshold, o.ddc_threshold, o.pmisr_max_rounds, o.poly_order) == (0.5, 0.9, 3, 6)
    assert (o.drop_R, o.drop_A, o.coarse_poly_order, o.coarse_iters, o.up_smooths) == (0.01, 0.001, 12, 3, 2)
    assert L.airg_status_string(-2).decode() == "malformed CSR matrix"


def test_struct_layouts_match_the_header():
    """Compile a tiny C program printing sizeof/offsetof and compare."""
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "airg.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(airg_opts), offsetof(airg_opts, seed),
         offsetof(airg_opts, device_bytes_cap), sizeof(airg_solve_info), sizeof(airg_level_info),
         sizeof(airg_stats), offsetof(airg_stats, vcycle_bytes_fp64));
  return 0;
}
"""
    tmp = tempfile.mkdtemp()
    c = os.path.join(tmp, "layout_probe.c")
    exe = os.path.join(tmp, "layout_probe")
    with open(c, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
    vals = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [C.sizeof(airg.Opts), airg.Opts.seed.offset, airg.Opts.device_bytes_cap.offset,
            C.sizeof(airg.SolveInfo), C.sizeof(airg.LevelInfo), C.sizeof(airg.Stats),
            airg.Stats.vcycle_bytes_fp64.offset]
    assert vals == want


def test_setup_rejects_null_arguments_on_host():
    """Argument checks run before any device work."""
    out = C.c_void_p()
    st = airg.lib().airg_setup(None, 4, 4, None, None, None, 1, None, None, None, C.byref(out))
    assert st == -1 and not out.value
    assert "null" in airg.lib().airg_last_error().decode()
