"""include/dock.h is plain C: a C99 program that includes it compiles with
gcc (-Wall -Werror -pedantic), links against the built library and calls it
(calls that need no GPU: the ABI version, host-side ligand preparation and
its validation)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_2410_10447_amd")

PROGRAM = r"""
#include <stdio.h>
#include "dock.h"

int main(void) {
    /* a 4-atom chain, the middle bond rotatable, an 8-class force field */
    double xyz[12] = {0, 0, 0, 1.5, 0, 0, 2.2, 1.3, 0, 3.7, 1.3, 0};
    double charge[4] = {0.1, -0.2, 0.15, -0.05};
    int32_t cls[4] = {0, 1, 2, 3};
    int32_t bonds[6] = {0, 1, 1, 2, 2, 3};
    int32_t rot[1] = {1};
    double radius[8], eps[8], solv[8], vol[8];
    for (int i = 0; i < 8; ++i) { radius[i] = 1.9; eps[i] = 0.15; solv[i] = -0.001; vol[i] = 30.0; }
    dock_ff_params ff;
    ff.n_classes = 8; ff.radius = radius; ff.eps = eps; ff.solv = solv; ff.vol = vol;
    ff.donor[0] = 6; ff.donor[1] = 7; ff.acceptor[0] = 3; ff.acceptor[1] = 4;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) { ff.hb_r0[a][b] = 1.9; ff.hb_eps[a][b] = 5.0; }
    dock_ligand_desc d;
    d.n_atoms = 4; d.n_torsions = 1; d.root_atom = 0; d.n_bonds = 3;
    d.xyz = xyz; d.charge = charge; d.cls = cls; d.bonds = bonds; d.rot_bonds = rot; d.ff = &ff;
    dock_ligand* lig = NULL;
    int32_t st = dock_create_ligand(&d, &lig);
    dock_ligand_info info;
    if (st == DOCK_OK) st = dock_ligand_info_get(lig, &info);
    printf("abi %d status %d atoms %d genes %d\n", (int)dock_abi_version(), (int)st,
           st == DOCK_OK ? (int)info.n_atoms : -1, st == DOCK_OK ? (int)info.n_genes : -1);
    dock_destroy_ligand(lig);
    /* validation: a NULL description is rejected with a message */
    st = dock_create_ligand(NULL, &lig);
    printf("null %d %s\n", (int)st, dock_last_error());
    return 0;
}
"""


def test_header_compiles_as_c_and_links(tmp_path):
    gcc = shutil.which("gcc")
    lib = os.path.join(LIB_DIR, "libdockmi.so")
    if not gcc or not os.path.exists(lib):
        pytest.skip("gcc or the built library missing")
    src = tmp_path / "use_dock.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "use_dock"
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-I" + os.path.join(ROOT, "include"),
                        str(src), "-o", str(exe), "-L" + LIB_DIR, "-ldockmi", "-Wl,-rpath," + LIB_DIR],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.splitlines()
    from paper_2410_10447_amd import dock
    assert lines[0] == f"abi {dock.ABI_VERSION} status 0 atoms 4 genes 8", lines
    assert lines[1].startswith(f"null {dock.DOCK_EINVAL} ")
