// C wrapper over the host-only phase machine of the closed-loop ball task
// (csrc/episode.h), so that its rules are tested on the CPU.
#include "episode.h"

extern "C" int ep_run(int n, const double *obs, const double *rule, int *status, int *phase, double *times)
{
    const mppi::EpRule r = {rule[0], rule[1], rule[2], rule[3], rule[4], rule[5]};
    mppi::EpState s;
    for (int i = 0; i < n; ++i) {
        const double *o = obs + 6 * i;
        const mppi::EpObs ob = {o[0], o[1], o[2], o[3], o[4], (int)o[5]};
        status[i] = mppi::ep_step(s, r, ob);
        phase[i] = s.phase;
    }
    times[0] = s.t_switch;
    times[1] = s.t_end;
    return 0;
}
