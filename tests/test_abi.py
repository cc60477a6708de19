"""The C-ABI library loads, exports every function include/igmres.h declares,
and its ctypes mirrors have the C layouts (checked against gcc's view of the
header).  No compute call is made."""
import os
import re
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "igmres.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ["mdp_create", "mdp_destroy", "bellman_apply", "policy_eval_gmres",
                 "igmres_pi_solve", "pi_solve", "opi_solve", "ig_last_error"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2211_04299_amd import igmres
    out = subprocess.run(["nm", "-D", "--defined-only", igmres.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(igmres.EXPORTS) <= exported


def test_ctypes_layouts_match_c(tmp_path):
    from paper_2211_04299_amd import igmres
    import ctypes
    prog = tmp_path / "sz.c"
    prog.write_text(textwrap.dedent(f"""
        #include <stdio.h>
        #include <stddef.h>
        #include "{HEADER}"
        int main(void) {{
          printf("%zu %zu %zu %zu\\n", sizeof(ig_mdp_desc), sizeof(ig_params), sizeof(ig_stats),
                 sizeof(ig_mdp_info));
          printf("%zu %zu %zu\\n", offsetof(ig_mdp_desc, validate), offsetof(ig_params, engine),
                 offsetof(ig_stats, alg_bytes));
          return 0;
        }}"""))
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", str(prog), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in lines[0].split()]
    assert sizes == [ctypes.sizeof(igmres.MdpDesc), ctypes.sizeof(igmres.Params),
                     ctypes.sizeof(igmres.Stats), ctypes.sizeof(igmres.MdpInfo)]
    offs = [int(x) for x in lines[1].split()]
    assert offs == [igmres.MdpDesc.validate.offset, igmres.Params.engine.offset,
                    igmres.Stats.alg_bytes.offset]


def test_params_default_is_theorem1_midpoint():
    from paper_2211_04299_amd import igmres
    p = igmres.params_default(0.99)
    assert p.alpha == pytest.approx(0.5 * 0.01 / 1.99)
    assert p.restart == 30 and p.tol == 1e-8 and p.mode == igmres.IG_MODE_FP64
