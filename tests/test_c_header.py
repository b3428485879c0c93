"""include/mpm.h, mpm_fem.h and mpm_rb.h are C headers: a C99 program includes
them, links libmpmx.so, and exercises the argument checks (no device needed)."""
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
#include "mpm_fem.h"
#include "mpm_rb.h"

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
  /* FEM: a description with too few nodes is refused before any allocation */
  mpm_fem_desc fd;
  memset(&fd, 0, sizeof fd);
  fd.n_envs = 1; fd.n_nodes = 3; fd.n_tets = 1; fd.dt = 1e-4f;
  int32_t tet[4] = {0, 1, 2, 3};
  mpm_fem* f = NULL;
  if (mpm_fem_create(&fd, tet, NULL, NULL, &f) != MPM_INVALID_ARG || f != NULL) return 6;
  if (mpm_fem_forward(NULL, 1, NULL, 0) != MPM_INVALID_ARG) return 7;
  /* rigid bodies: link 1 names itself as its parent, which is refused */
  mpm_rb_link links[2];
  memset(links, 0, sizeof links);
  for (int i = 0; i < 2; ++i) {
    links[i].parent = i - 1;
    links[i].joint_rot[0] = links[i].joint_rot[4] = links[i].joint_rot[8] = 1.f;
    links[i].axis[0] = 1.f;
    links[i].mass = 1.f;
  }
  links[1].parent = 1;
  mpm_rb_desc rd;
  memset(&rd, 0, sizeof rd);
  rd.n_envs = 1; rd.n_links = 2; rd.max_substeps = 1; rd.dt = 1e-3f; rd.gravity[2] = -9.8f;
  mpm_rb* r = NULL;
  if (mpm_rb_create(&rd, links, NULL, NULL, NULL, &r) != MPM_INVALID_ARG || r != NULL) return 8;
  if (mpm_rb_backward(NULL, NULL, NULL, NULL, NULL, NULL, NULL) != MPM_INVALID_ARG) return 9;
  if (MPM_RB_PARAMS != 5 || MPM_FEM_PARAMS != 8) return 10;
  /* several colliders per env: the indexed setters check their handle first */
  const float c3[3] = {0.5f, 0.5f, 0.5f};
  if (MPM_MAX_COLLIDERS < 2 || mpm_set_collider(NULL, 0, 1, MPM_COLLIDER_BOX, c3, c3, 0.f, c3, 10.f, 0.1f) !=
      MPM_INVALID_ARG) return 11;
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
