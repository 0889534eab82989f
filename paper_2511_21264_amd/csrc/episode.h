// Phase machine and termination rules of the closed-loop ball transport
// (Sec. IV-B: pick and move phases switch the cost terms on and off; the
// experiments' success metric: a run fails on a collision, on a timeout or
// when the ball falls).  Host-only, so the rules are tested on the CPU.
//
// Readings (the paper names the phases and failure causes, not the tests):
//   * pick -> move when the pad midpoint is within grasp_tol of the grasp
//     point p_ball - (0, 0, eps) and the pad distance within width_tol of
//     l_ball, at the state after an executed control step;
//   * collision: some arm-arm or arm-box pair at negative signed distance
//     after an executed step;
//   * the ball has fallen when, in the move phase and after it has been
//     above lift_z, it is below drop_z;
//   * success: in the move phase, the ball within goal_tol of the goal;
//   * timeout: the simulated time reaches t_max with none of the above.
// Checks run in this order after every executed step; the first outcome
// other than "running" ends the run.
#pragma once

namespace mppi {

enum EpStatus { EP_RUNNING = 0, EP_SUCCESS = 1, EP_FAIL_COLLISION = -1, EP_FAIL_TIMEOUT = -2, EP_FAIL_DROP = -3 };
enum EpPhase { EP_PICK = 0, EP_MOVE = 1 };

struct EpRule {
    double grasp_tol, width_tol, goal_tol, lift_z, drop_z, t_max;
};

// what one executed control step shows (post-step state)
struct EpObs {
    double t;           // simulated time after the step (s)
    double goal_dist;   // |p_ball - p_goal|
    double grasp_dist;  // |c - (p_ball - (0, 0, eps))|, c the pad midpoint
    double width_err;   // | |p1 - p2| - l_ball |
    double ball_z;
    int penetrations;   // arm-arm and arm-box pairs at negative distance
};

struct EpState {
    int phase = EP_PICK;
    int status = EP_RUNNING;
    int lifted = 0;
    double t_switch = -1.0;  // time of the pick -> move switch (-1: none)
    double t_end = -1.0;     // time of the outcome (-1: running)
};

inline int ep_step(EpState &s, const EpRule &r, const EpObs &o)
{
    if (s.status != EP_RUNNING) return s.status;
    if (o.penetrations > 0) {
        s.status = EP_FAIL_COLLISION;
    } else if (s.phase == EP_PICK) {
        if (o.grasp_dist < r.grasp_tol && o.width_err < r.width_tol) {
            s.phase = EP_MOVE;
            s.t_switch = o.t;
        }
    } else {
        if (o.ball_z > r.lift_z) s.lifted = 1;
        if (s.lifted && o.ball_z < r.drop_z)
            s.status = EP_FAIL_DROP;
        else if (o.goal_dist < r.goal_tol)
            s.status = EP_SUCCESS;
    }
    if (s.status == EP_RUNNING && o.t >= r.t_max) s.status = EP_FAIL_TIMEOUT;
    if (s.status != EP_RUNNING) s.t_end = o.t;
    return s.status;
}

}  // namespace mppi
