"""State-space selection (oracle; test infrastructure).

Paper passage followed: Sec. III.B, the algorithm of Fig. 2 (construction,
solving, calculation of each state's probability growth speed, comparison
with a preset epsilon, deletion, normalisation, repeat until t_f) and the
sizes of Table I.

Readings of what the paper leaves open:

* Growth speed of state s over one solve of k steps of length dt:
  |p_s(after) - p_s(before)| / (k dt), an absolute rate of change (states
  whose probability neither grows nor decays do not take part in the
  dynamics).  A state is deleted when its speed is below epsilon, so
  epsilon = 0 deletes nothing.
* "Normalised": the kept block P rho P is rescaled to the trace the state had
  before the deletion (1 - sink); the sink is carried unchanged.
* The next solve runs on the kept states: H and the decoherence operators
  are restricted to them (P H P, P A P), while A^dag A is taken before the
  projection, so probability that a decoherence operator moves onto a
  deleted state leaves through the sink, as for the excitation window.
* The next comparison starts from the renormalised state.
* Deleted states never return.
"""
from __future__ import annotations

import numpy as np

from . import evolve


def growth_speed(p_before, p_after, interval):
    """|p_after - p_before| / interval, per state."""
    return np.abs(np.asarray(p_after) - np.asarray(p_before)) / float(interval)


def select_evolve(wl, rho0, n_steps, eps, every=1, sink0=0.0):
    """The selection loop for n_steps steps, comparing after every `every`
    steps.  Returns (rho, sink, kept, sizes): the final reduced state, its
    sink, the indices of its states in the window basis and the basis size
    after each solve."""
    general = bool(wl.get("general", False))
    sysm = evolve.GeneralSystem(wl) if general else evolve.System(wl)
    kept = np.arange(sysm.n)
    rho, sink = np.asarray(rho0, dtype=np.complex128), float(sink0)
    sizes = []
    done = 0
    while done < n_steps:
        k = min(every, n_steps - done)
        p_before = np.real(np.diag(rho)).copy()
        for _ in range(k):
            rho, sink = evolve.step(rho, sink, sysm.u, sysm.jumps, sysm.dt)
        done += k
        speed = growth_speed(p_before, np.real(np.diag(rho)), k * sysm.dt)
        sel = np.nonzero(speed >= eps)[0]
        if sel.size == 0:
            raise ValueError("every state would be removed")
        if sel.size < sysm.n:
            block = rho[np.ix_(sel, sel)]
            rho = block * ((1.0 - sink) / np.trace(block).real)
            kept = kept[sel]
            sysm = (evolve.GeneralSystem(wl, keep=kept) if general
                    else evolve.System(wl, occ=sysm.occ[sel]))
        sizes.append(sysm.n)
    return rho, sink, kept, sizes
