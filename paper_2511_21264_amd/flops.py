"""Algorithmic FP32 work model of the rollout kernel.

Counts are of the arithmetic the rollout algorithm performs per unit of
work (an FMA counts 2, add/mul/min/max/compare 1, sqrt/div/sin/cos/log 1),
hand-counted from the stage definitions:

  per physics substep (free space, both arms + ball):
    PD target and torques      182     FK (2 arms, 7 joints)        336
    composite-body inertia    2884     Cholesky (2 x 7x7)           294
    Newton-Euler bias         2462     free-velocity solves         196
    free velocity, ball, integration and quaternion update          124
    -> F_FREE = 6478
  broadphase: AABBs of the 15 moving geoms 180 + 6 compares per candidate pair
  narrowphase: 60 per evaluated pair, capsule-box 1350 (two bisections)
  contact rows: 1120 per contact (point Jacobian, Mt^-1 J^T, 3x3 block,
    pyramid edges, diagonal)
  Gauss-Seidel: 363 per contact per sweep (4 rows)
  per control step cost: FK 336 + stage terms 92 + AABBs 168 + 6 per cost
    pair compare + 5 per cost pair term
  box-shaped object, per substep: rotation from the quaternion 30, world
    inverse inertia 72, gyroscopic step 51, rotated AABB 27, the eight
    vertex heights against the table 150 -> F_BOX_FREE = 330 (its pair
    tests are counted at the narrowphase rates above: a lower bound)
  further task terms, per control step: joint deviation 42, vertical 2,
    pad velocities and relative velocity 200, position / x targets 24,
    orientation angles 2 x 60 + 40 -> F_EXT = 428
"""

F_FREE = 6478
F_AABB = 180
F_BP_PAIR = 6
F_NP = 60
F_NP_BOX = 1350
F_ROWS = 1120
F_PGS = 363
F_COST_FIXED = 336 + 92 + 168
F_COST_PAIR = 11
F_BOX_FREE = 330
F_EXT = 428


def rollout_flops(K, H, n_sub, n_pairs, n_cost_pairs, n_pgs, contacts, np_tests, box_tests, obj_box=False,
                  ext=False):
    """Algorithmic FP32 operations of one rollout launch.

    contacts / np_tests / box_tests are the launch's totals reported by the
    library (sums over samples and substeps; np_tests includes the cost's
    distance evaluations and box_tests the capsule-box ones among them).
    """
    n_substeps = K * H * n_sub
    n_steps = K * H
    f = n_substeps * (F_FREE + F_AABB + F_BP_PAIR * n_pairs)
    f += contacts * (F_ROWS + n_pgs * F_PGS)
    f += (np_tests - box_tests) * F_NP + box_tests * F_NP_BOX
    f += n_steps * (F_COST_FIXED + F_COST_PAIR * n_cost_pairs)
    if obj_box:
        f += n_substeps * F_BOX_FREE
    if ext:
        f += n_steps * F_EXT
    return float(f)
