"""include/mpm.h is a C header: a C99 program includes it, links libmpmx.so,
and exercises the argument checks (no device needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_2412_12089_amd")

C_SRC = r"""
#include <stdio.h>
#include <string.h>
#include "mpm.h"

int main(void) {
  mpm_env_desc env;
  memset(&env, 0, sizeof env);
  env.n = 30;                 /* not a multiple of 4 */
  env.material = MPM_COROTATED;
  env.n_particles = 10;
  env.dt = 1e-4f;
  env.wall = 3;
  mpm_batch_desc d;
  memset(&d, 0, sizeof d);
  d.n_envs = 1; d.envs = &env; d.max_substeps = 4; d.ckpt_every = 2; d.mode = MPM_MODE_BATCHED;
  mpm_batch* b = NULL;
  int rc = mpm_batch_create(&d, NULL, NULL, &b);
  if (rc != MPM_INVALID_ARG || b != NULL) return 1;
  if (mpm_forward(NULL, 1, MPM_FWD_RECORD) != MPM_INVALID_ARG) return 2;
  if (mpm_backward(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) != MPM_INVALID_ARG) return 3;
  if (mpm_set_option(NULL, MPM_OPT_P2G, 1) != MPM_INVALID_ARG) return 4;
  if (strncmp(mpm_version(), "mpmx", 4) != 0) return 5;
  printf("ok %s\n", mpm_version());
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_header_is_c99_and_links(tmp_path):
    lib = os.path.join(LIB_DIR, "libmpmx.so")
    assert os.path.exists(lib), "build the library first"
    src = tmp_path / "use_mpm.c"
    src.write_text(C_SRC)
    exe = tmp_path / "use_mpm"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-L", LIB_DIR, "-lmpmx", "-Wl,-rpath," + LIB_DIR, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, (out.returncode, out.stderr)
    assert out.stdout.startswith("ok mpmx")
