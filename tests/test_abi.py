"""The C-ABI library loads, exports every function include/igmres.h declares,
and its ctypes mirrors have the C layouts (checked against gcc's view of the
header).  No compute call is made."""
import os
import re
import subprocess

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
    """Size of every mirrored struct and the offset of every field."""
    from paper_2211_04299_amd import igmres
    import ctypes
    pairs = [("ig_mdp_desc", igmres.MdpDesc), ("ig_params", igmres.Params),
             ("ig_stats", igmres.Stats), ("ig_mdp_info", igmres.MdpInfo),
             ("ig_server_config", igmres.ServerConfig), ("ig_server_info", igmres.ServerInfo)]
    body = []
    for cname, py in pairs:
        body.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            body.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    prog = tmp_path / "sz.c"
    prog.write_text("#include <stdio.h>\n#include <stddef.h>\n"
                    f'#include "{HEADER}"\n'
                    "int main(void) {\n" + "\n".join(body) + "\nreturn 0;\n}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", str(prog), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for _, py in pairs:
        want.append(ctypes.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert got == want


def test_params_default_is_theorem1_midpoint():
    from paper_2211_04299_amd import igmres
    p = igmres.params_default(0.99)
    assert p.alpha == pytest.approx(0.5 * 0.01 / 1.99)
    assert p.restart == 30 and p.tol == 1e-8 and p.mode == igmres.IG_MODE_FP64
    assert p.forcing == 0 and p.polish == 0 and p.precond == 0 and p.engine == 0
