"""The C ABI header is plain C: it compiles as strict C99 (gcc -pedantic, no C++), and a C program
links against libfe.so and calls an entry point that needs no GPU (argument checking)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2605_08523_amd")

C_SOURCE = r"""
#include "fe.h"
#include <stdio.h>
#include <string.h>
int main(void) {
    /* argument checking needs no device: a NULL output is refused with a message */
    int rc = fe_workspace_create(256, 0, 0, NULL);
    if (rc != FE_ERR_ARG) return 1;
    if (strlen(fe_last_error()) == 0) return 2;
    printf("ok %d\n", rc);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_c99_and_links(tmp_path):
    src = tmp_path / "abi.c"
    src.write_text(C_SOURCE)
    obj = tmp_path / "abi.o"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o", str(obj)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    if not os.path.exists(os.path.join(PKG, "libfe.so")):
        pytest.fail("libfe.so is not built (python -m paper_2605_08523_amd.build)")
    exe = tmp_path / "abi"
    r = subprocess.run(["gcc", str(obj), "-L", PKG, "-lfe", f"-Wl,-rpath,{PKG}", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.returncode, r.stdout, r.stderr)
