"""The C-ABI library loads (no GPU needed) and exports every function that
include/mppi.h declares; the binding's scene marshalling matches the header."""
import ctypes as C
import os
import re

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mppi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mppi_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    import paper_2511_21264_amd as mp
    L = mp.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def test_binding_declares_the_same_entry_points():
    import paper_2511_21264_amd as mp
    src = open(mp.__file__).read()
    for n in _declared():
        assert f'"{n}"' in src, n


def test_desc_struct_layout_matches_header():
    """Offsets of a few fields computed by the C compiler equal the ctypes ones."""
    import subprocess
    import tempfile
    import paper_2511_21264_amd as mp
    code = r'''
#include <stddef.h>
#include <stdio.h>
#include "mppi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(mppi_scene_desc), offsetof(mppi_scene_desc, n_box),
         offsetof(mppi_scene_desc, goal), offsetof(mppi_scene_desc, n_cmax), offsetof(mppi_scene_desc, eps_frac),
         sizeof(mppi_stats));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    D = mp.SceneDesc
    want = [C.sizeof(D), D.n_box.offset, D.goal.offset, D.n_cmax.offset, D.eps_frac.offset, C.sizeof(mp.Stats)]
    assert [int(v) for v in out] == want


def test_request_and_server_struct_layouts_match_header():
    import subprocess
    import tempfile
    import paper_2511_21264_amd as mp
    code = r'''
#include <stddef.h>
#include <stdio.h>
#include "mppi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mppi_request),
         offsetof(mppi_request, lambda), offsetof(mppi_request, opts), offsetof(mppi_request, U_new),
         offsetof(mppi_request, status), sizeof(mppi_server_opts), offsetof(mppi_server_opts, flags),
         sizeof(mppi_ticket_info), offsetof(mppi_ticket_info, t_done_ms), sizeof(mppi_server_info),
         offsetof(mppi_server_info, mem_high_water), offsetof(mppi_server_info, pending), sizeof(mppi_opts));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    R, O, T, I = mp.Request, mp.ServerOpts, mp.TicketInfo, mp.ServerInfo
    want = [C.sizeof(R), R.lam.offset, R.opts.offset, R.U_new.offset, R.status.offset, C.sizeof(O), O.flags.offset,
            C.sizeof(T), T.t_done_ms.offset, C.sizeof(I), I.mem_high_water.offset, I.pending.offset,
            C.sizeof(mp.Opts)]
    assert [int(v) for v in out] == want


def test_qp_struct_layout_matches_header():
    import subprocess
    import tempfile
    import paper_2511_21264_amd as mp
    code = r'''
#include <stddef.h>
#include <stdio.h>
#include "mppi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(mppi_qp), offsetof(mppi_qp, pos_hi), offsetof(mppi_qp, acc_max),
         offsetof(mppi_qp, rho), offsetof(mppi_qp, alpha), offsetof(mppi_qp, iters));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    Q = mp.QP
    assert [int(v) for v in out] == [C.sizeof(Q), Q.pos_hi.offset, Q.acc_max.offset, Q.rho.offset, Q.alpha.offset,
                                     Q.iters.offset]


def test_cov_struct_layout_and_constants_match_header():
    import subprocess
    import tempfile
    import paper_2511_21264_amd as mp
    code = r'''
#include <stddef.h>
#include <stdio.h>
#include "mppi.h"
int main(void) {
  printf("%zu %zu %zu %zu %d %d\n", sizeof(mppi_cov), offsetof(mppi_cov, Sigma_out), offsetof(mppi_cov, eps),
         offsetof(mppi_cov, U_best), MPPI_COV_MAX_N, MPPI_E_NOTPD);
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    V = mp.Cov
    assert [int(v) for v in out] == [C.sizeof(V), V.Sigma_out.offset, V.eps.offset, V.U_best.offset, mp.COV_MAX_N,
                                     mp.E_NOTPD]


def test_episode_struct_layouts_match_header():
    import subprocess
    import tempfile
    import paper_2511_21264_amd as mp
    code = r'''
#include <stddef.h>
#include <stdio.h>
#include "mppi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mppi_episode_opts), offsetof(mppi_episode_opts, grasp_tol),
         offsetof(mppi_episode_opts, t_max), offsetof(mppi_episode_opts, cov_eps), sizeof(mppi_episode_result),
         offsetof(mppi_episode_result, t_end), offsetof(mppi_episode_result, ball_final),
         offsetof(mppi_episode_result, n_diverged));
  return 0;
}'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(code)
        exe = os.path.join(d, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    E, R = mp.EpisodeOpts, mp.EpisodeResult
    assert [int(v) for v in out] == [C.sizeof(E), E.grasp_tol.offset, E.t_max.offset, E.cov_eps.offset, C.sizeof(R),
                                     R.t_end.offset, R.ball_final.offset, R.n_diverged.offset]


def test_scene_desc_roundtrip():
    import paper_2511_21264_amd as mp
    sc = W.make_scene(3)
    d = mp.scene_desc(sc)
    assert d.n_box == sc["n_box"] == 8
    assert np.allclose(np.array(d.box_c[:24]).reshape(8, 3), sc["box_c"])
    assert d.n_cmax == sc["n_cmax"]
