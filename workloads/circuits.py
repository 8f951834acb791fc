"""Cut circuits: gate lists, wire cuts and the subcircuits they define.

A circuit is a list of one-qubit unitaries and CZ gates on ``n_qubits``
wires.  A cut ``(q, pos)`` severs wire ``q`` between the gates with op index
``<= pos`` and those after it (Section 3.1: cuts are timewise, on qubit
wires).  Each wire is thereby split into segments; a cut solution assigns
every segment to a subcircuit, and every two-qubit gate must stay inside one
subcircuit (Section 4.1: cuts are the cross-cluster edges of the circuit
DAG).

Conventions used by every consumer of these structures:

* Cut ids are the positions of the cuts sorted by ``(qubit, pos)``.
* A subcircuit's register slots are its segments sorted by
  ``(qubit, segment)``.  Slot 0 is the most significant bit of the
  subcircuit's outcome index.
* ``init_cut[s]`` is the id of the cut whose downstream end starts slot
  ``s`` (the slot is initialised by the cut), else -1.  ``meas_cut[s]`` is
  the id of the cut whose upstream end closes slot ``s`` (the slot is
  measured for the cut), else -1.  Slots with ``meas_cut == -1`` carry the
  subcircuit's outputs.
* ``out_perm[i]`` is the uncut-circuit qubit carried by bit ``i`` of the
  concatenated output index (subcircuit 0's outputs most significant, slot
  order inside each subcircuit).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Op:
    """One gate: ``name`` is ``'u'`` (2x2 unitary ``matrix``) or ``'cz'``."""

    name: str
    qubits: tuple
    matrix: np.ndarray | None = None


@dataclass
class SubcircuitSpec:
    """One subcircuit: its slots, cut roles and gates (in slot indices)."""

    width: int
    init_cut: list
    meas_cut: list
    slots: list                  # (qubit, segment) per slot
    ops: list = field(default_factory=list)  # Op with slot indices


@dataclass
class CutCircuit:
    n_qubits: int
    ops: list
    cuts: list                   # (qubit, pos), sorted; index = cut id
    assignment: dict             # (qubit, segment) -> subcircuit id

    def __post_init__(self):
        self.cuts = sorted(self.cuts)
        if len(set(self.cuts)) != len(self.cuts):
            raise ValueError("duplicate cut")
        self._check()

    # -- segments ---------------------------------------------------------
    def n_segments(self, q: int) -> int:
        return 1 + sum(1 for (cq, _) in self.cuts if cq == q)

    def segment(self, q: int, op_index: int) -> int:
        return sum(1 for (cq, pos) in self.cuts if cq == q and pos < op_index)

    @property
    def n_subcircuits(self) -> int:
        return 1 + max(self.assignment.values())

    def _check(self):
        for q in range(self.n_qubits):
            for s in range(self.n_segments(q)):
                if (q, s) not in self.assignment:
                    raise ValueError(f"segment {(q, s)} not assigned")
        for i, op in enumerate(self.ops):
            subs = {self.assignment[(q, self.segment(q, i))] for q in op.qubits}
            if len(subs) != 1:
                raise ValueError(f"op {i} {op.name}{op.qubits} crosses subcircuits")
        for cid, (q, pos) in enumerate(self.cuts):
            s = self.segment(q, pos + 1) - 1
            up, down = self.assignment[(q, s)], self.assignment[(q, s + 1)]
            if up == down:
                raise ValueError(f"cut {cid} joins a subcircuit to itself")

    # -- derived structures ----------------------------------------------
    def cut_ends(self, cid: int):
        """(upstream subcircuit, downstream subcircuit) of cut ``cid``."""
        q, pos = self.cuts[cid]
        s = self.segment(q, pos + 1) - 1
        return self.assignment[(q, s)], self.assignment[(q, s + 1)]

    def subcircuits(self) -> list:
        out = []
        for c in range(self.n_subcircuits):
            slots = sorted(k for k, v in self.assignment.items() if v == c)
            index = {k: i for i, k in enumerate(slots)}
            init_cut, meas_cut = [-1] * len(slots), [-1] * len(slots)
            for cid, (q, pos) in enumerate(self.cuts):
                s = self.segment(q, pos + 1) - 1
                if (q, s) in index:
                    meas_cut[index[(q, s)]] = cid
                if (q, s + 1) in index:
                    init_cut[index[(q, s + 1)]] = cid
            ops = []
            for i, op in enumerate(self.ops):
                keys = [(q, self.segment(q, i)) for q in op.qubits]
                if keys[0] in index:
                    ops.append(Op(op.name, tuple(index[k] for k in keys), op.matrix))
            out.append(SubcircuitSpec(len(slots), init_cut, meas_cut, slots, ops))
        return out

    def out_perm(self) -> list:
        perm = []
        for spec in self.subcircuits():
            for (q, s), m in zip(spec.slots, spec.meas_cut):
                if m == -1:
                    perm.append(q)
        return perm


# ---------------------------------------------------------------------------
# Random gates
# ---------------------------------------------------------------------------

def haar_u2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 2x2 unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))


H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2.0)
XGATE = np.array([[0, 1], [1, 0]], dtype=complex)


def masked_brickwork(n: int, layers: int, cut_layers, assign, seed: int) -> CutCircuit:
    """Brickwork of ``layers`` layers on a line: each layer applies a
    Haar-random one-qubit unitary to every qubit, then CZ(i, i+1) for every
    i with i = t (mod 2).  ``cut_layers`` lists (qubit, t): cut the wire
    after layer t.  ``assign(q, segment) -> subcircuit``.  A CZ whose two
    wire segments fall in different subcircuits is dropped, which makes the
    circuit separable by the given cuts (the uncut reference circuit is the
    same masked circuit, simulated whole)."""
    rng = np.random.default_rng(seed)

    def seg(q, t):
        return sum(1 for (cq, ct) in cut_layers if cq == q and ct < t)

    ops, last_op_of_layer = [], []
    for t in range(layers):
        for q in range(n):
            ops.append(Op("u", (q,), haar_u2(rng)))
        for i in range(t % 2, n - 1, 2):
            if assign(i, seg(i, t)) == assign(i + 1, seg(i + 1, t)):
                ops.append(Op("cz", (i, i + 1)))
        last_op_of_layer.append(len(ops) - 1)
    cuts = [(q, last_op_of_layer[t]) for (q, t) in cut_layers]
    assignment = {}
    for q in range(n):
        for s in range(1 + sum(1 for (cq, _) in cut_layers if cq == q)):
            assignment[(q, s)] = assign(q, s)
    return CutCircuit(n, ops, cuts, assignment)


def two_way_circuit_8q(seed: int = 0) -> CutCircuit:
    """8 qubits, 5 brickwork layers, one cut on q4 after layer 2.
    Subcircuit 0: q0..q3 and q4 up to the cut (5 slots); subcircuit 1: q4
    after the cut and q5..q7 (4 slots)."""
    def assign(q, s):
        if q < 4:
            return 0
        if q == 4:
            return 0 if s == 0 else 1
        return 1
    return masked_brickwork(8, 5, [(4, 2)], assign, seed)


def two_way_circuit_20q(seed: int = 1) -> CutCircuit:
    """20 qubits, 10 brickwork layers, four cuts after layer 4: q8, q9 move
    from subcircuit 0 to 1 and q10, q11 from subcircuit 1 to 0, giving two
    subcircuits of 12 slots and 10 outputs each."""
    def assign(q, s):
        if q in (8, 9):
            return 0 if s == 0 else 1
        if q in (10, 11):
            return 1 if s == 0 else 0
        return 0 if q < 8 else 1
    return masked_brickwork(20, 10, [(8, 4), (9, 4), (10, 4), (11, 4)], assign, seed)


def two_way_circuit_30q(seed: int = 3, layers: int = 8) -> CutCircuit:
    """30 qubits, ``layers`` brickwork layers, four cuts after layer 3: q12,
    q13 move from subcircuit 0 to 1 and q14, q15 from subcircuit 1 to 0,
    giving subcircuits of 16 slots (14 outputs) and 18 slots (16 outputs)."""
    def assign(q, s):
        if q in (12, 13):
            return 0 if s == 0 else 1
        if q in (14, 15):
            return 1 if s == 0 else 0
        return 0 if q < 12 else 1
    return masked_brickwork(30, layers, [(12, 3), (13, 3), (14, 3), (15, 3)], assign, seed)


def cut_circuit_from_clusters(n: int, ops, cluster) -> CutCircuit:
    """The cut circuit that a clustering of the two-qubit gates defines:
    ``cluster[g]`` is the subcircuit of the g-th two-qubit gate of ``ops``.
    A wire is cut right after a two-qubit gate whose next two-qubit gate on
    that wire lies in another cluster; every wire segment belongs to the
    cluster of the two-qubit gates it holds (a segment before a wire's first
    two-qubit gate to that gate's cluster)."""
    two = [i for i, op in enumerate(ops) if len(op.qubits) == 2]
    if len(two) != len(cluster):
        raise ValueError("one cluster label per two-qubit gate")
    label = dict(zip(two, cluster))
    cuts, assignment = [], {}
    for q in range(n):
        on_q = [i for i in two if q in ops[i].qubits]
        if not on_q:
            raise ValueError(f"qubit {q} takes part in no two-qubit gate")
        seg = 0
        assignment[(q, 0)] = label[on_q[0]]
        for a, b in zip(on_q, on_q[1:]):
            if label[a] != label[b]:
                cuts.append((q, a))
                seg += 1
                assignment[(q, seg)] = label[b]
    return CutCircuit(n, list(ops), cuts, assignment)


def hidden_string_circuit(secret, groups) -> CutCircuit:
    """Bernstein-Vazirani hidden-string circuit (Section 5.3 lists it as a
    sparse-output benchmark) written from the algorithm's definition.
    Data qubits 0..n-1, ancilla n.  The ancilla starts in |1>, all qubits get
    H, every data qubit i with secret bit 1 drives CNOT(i -> ancilla) (built
    as H CZ H on the ancilla), then H on every qubit.  The output is the
    single basis state (secret, 1) with probability 1.

    ``groups`` partitions the data qubits into consecutive runs; the ancilla
    wire is cut between runs so that subcircuit g holds run g and the
    ancilla segment that talks to it (a chain of len(groups) subcircuits)."""
    n = len(secret)
    anc = n
    ops = [Op("u", (anc,), XGATE)]
    ops += [Op("u", (q,), H) for q in range(n + 1)]
    cuts = []
    group_of = {}
    for g, run in enumerate(groups):
        for q in run:
            group_of[q] = g
        for q in run:
            if secret[q]:
                ops.append(Op("u", (anc,), H))
                ops.append(Op("cz", (q, anc)))
                ops.append(Op("u", (anc,), H))
        if g + 1 < len(groups):
            cuts.append((anc, len(ops) - 1))
    ops += [Op("u", (q,), H) for q in range(n + 1)]
    assignment = {(q, 0): group_of[q] for q in range(n)}
    for s in range(len(groups)):
        assignment[(anc, s)] = s
    return CutCircuit(n + 1, ops, cuts, assignment)


def random_cut_circuit(rng: np.random.Generator, n: int, n_sub: int, n_cuts: int,
                       depth: int):
    """A random small cut circuit: wires are split by ``n_cuts`` cuts at
    random positions, segments are assigned to ``n_sub`` subcircuits at
    random (consecutive segments of a wire always differ), then ``depth``
    rounds of random one-qubit unitaries and random CZs between segments
    that are alive at the same time in the same subcircuit are laid down.
    Returns None when the draw leaves a subcircuit empty."""
    # cut times on a discrete clock 1..depth-1
    cut_times = {}
    for _ in range(n_cuts):
        q = int(rng.integers(n))
        t = int(rng.integers(1, depth))
        cut_times.setdefault(q, set()).add(t)
    cut_list = sorted((q, t) for q, ts in cut_times.items() for t in ts)
    assign = {}
    for q in range(n):
        ts = sorted(cut_times.get(q, ()))
        prev = None
        for s in range(len(ts) + 1):
            choices = [c for c in range(n_sub) if c != prev]
            c = int(rng.choice(choices))
            assign[(q, s)] = c
            prev = c
    if set(assign.values()) != set(range(n_sub)):
        return None

    def seg(q, t):
        return sum(1 for tt in cut_times.get(q, ()) if tt <= t)

    ops, cut_pos = [], {}
    for t in range(depth):
        # a cut at time t sits before the gates of round t
        for q in range(n):
            if t in cut_times.get(q, ()):
                cut_pos[(q, t)] = len(ops) - 1
        for q in range(n):
            ops.append(Op("u", (q,), haar_u2(rng)))
        order = rng.permutation(n)
        used = set()
        for a in order:
            if a in used:
                continue
            partners = [b for b in range(n) if b != a and b not in used
                        and assign[(b, seg(b, t))] == assign[(a, seg(a, t))]]
            if partners and rng.random() < 0.8:
                b = int(rng.choice(partners))
                used.update((int(a), b))
                ops.append(Op("cz", (int(a), b)))
    for q in range(n):
        ops.append(Op("u", (q,), haar_u2(rng)))
    cuts = [(q, cut_pos[(q, t)]) for (q, t) in cut_list]
    return CutCircuit(n, ops, cuts, assign)
