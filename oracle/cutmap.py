"""Facts the oracle reads off a subcircuit's cut map.

A subcircuit is given as (width, init_cut, meas_cut): per register slot, the
cut id that initialises it or -1, and the cut id it is measured for or -1
(Section 3.1: a cut splits a wire into an upstream piece that is measured
and a downstream piece that is initialised).
"""
from __future__ import annotations


def unpack(sub):
    """Accept a (width, init_cut, meas_cut) tuple or an object with those
    attributes."""
    if isinstance(sub, tuple):
        return sub
    return sub.width, list(sub.init_cut), list(sub.meas_cut)


def outputs(sub):
    """Slots that are measured as circuit outputs (not for a cut)."""
    w, _, meas = unpack(sub)
    return [s for s in range(w) if meas[s] == -1]


def init_slots(sub):
    w, init, _ = unpack(sub)
    return [s for s in range(w) if init[s] != -1]


def meas_slots(sub):
    w, _, meas = unpack(sub)
    return [s for s in range(w) if meas[s] != -1]


def incident_cuts(sub):
    """Cut ids touching the subcircuit, ascending: the digit order of its
    label index (first = most significant)."""
    _, init, meas = unpack(sub)
    return sorted({c for c in init + meas if c != -1})


def total_cuts(subs):
    ids = set()
    for s in subs:
        ids.update(incident_cuts(s))
    return len(ids)


def local_label(sub, global_digits):
    """Row of the subcircuit's entry tensor for a global labeling given as
    one digit (I=0, X=1, Y=2, Z=3) per cut id."""
    row = 0
    for c in incident_cuts(sub):
        row = 4 * row + global_digits[c]
    return row
