"""Policy and adjoint summaries that do not depend on how exact ties between
equivalent hosts are broken (oracle; test only).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

Every host has the same capacity and rates (Sec. V-B..V-D as read in
``oracle.model``), so permuting the hosts maps the chain onto itself and
V*(sigma n, e) = V*(n, e).  Two placements on hosts a, b with n_a = n_b then
have equal Q (their post-decision occupancies are permutations of each
other), and the lowest-index tie-break of Alg. 3 step 4 may pick either one
when the values are rounded.  The quantities below are the same for every
such choice:

* ``target_load``: the occupancy n_a of the host a policy places on (-1 for
  the paid cloud).  Where the best action is unique this is equivalent to the
  action itself; where it is tied only with equivalent hosts it is the
  common value.
* ``ambiguous``: the states where the best Q and the best Q over actions of a
  *different* target load are within a relative gap (those are genuine near
  ties, which rounding may resolve either way).
* ``orbit_sum``: a vector summed over each host-permutation orbit of states
  (the occupancy digits sorted, same class).  Routing a tie to an equivalent
  host moves discounted occupation mass between states of one orbit only, so
  the orbit sums of the adjoint weights w = (I - gamma P_pi)^-T c are the
  same for every tie routing of one target-load policy.
"""
from __future__ import annotations

import hashlib
from typing import Optional

import numpy as np

from . import vi


def target_load(p, pi: np.ndarray, g: Optional[vi.Grid] = None) -> np.ndarray:
    """n_{pi(s)} for placements, -1 for the paid cloud (int8, one per state)."""
    g = g or vi.grid(p)
    pi = np.asarray(pi, dtype=np.int64).reshape(p.J, g.n_occ)
    out = np.full((p.J, g.n_occ), -1, dtype=np.int8)
    occ = np.arange(g.n_occ)
    for e in range(p.J):
        place = pi[e] < p.K
        out[e, place] = g.digits[occ[place], pi[e][place]]
    return out.reshape(-1)


def ambiguous(p, V: np.ndarray, rel: float = 1e-6, g: Optional[vi.Grid] = None) -> np.ndarray:
    """Indices of the states whose best Q is within rel * max(|Q1|, 1e-3
    ||V||_inf) of the best Q over actions with another target load."""
    g = g or vi.grid(p)
    Q = vi.q_table(p, V, g).reshape(p.J, g.n_occ, p.K + 1)
    tl = np.full((p.J, g.n_occ, p.K + 1), -1, dtype=np.int64)
    tl[:, :, :p.K] = g.digits[None, :, :]
    best_a = np.argmax(Q, axis=2)
    Q1 = np.take_along_axis(Q, best_a[..., None], axis=2)[..., 0]
    tl1 = np.take_along_axis(tl, best_a[..., None], axis=2)[..., 0]
    other = np.where(tl != tl1[..., None], Q, -np.inf)
    Q2 = other.max(axis=2)
    denom = np.maximum(np.abs(Q1), 1e-3 * np.max(np.abs(V)))
    amb = (Q1 - Q2) <= rel * denom
    return np.flatnonzero(amb.reshape(-1))


def masked_digest(tl: np.ndarray, skip: np.ndarray) -> str:
    """SHA-256 of the target loads with the listed states set to -2."""
    t = np.array(tl, dtype=np.int8, copy=True)
    t[np.asarray(skip, dtype=np.int64)] = -2
    return hashlib.sha256(t.tobytes()).hexdigest()


def histogram(p, tl: np.ndarray) -> list:
    """Counts of each target load (-1..C) per class, [J][C+2]."""
    tl = np.asarray(tl, dtype=np.int64).reshape(p.J, -1)
    return [np.bincount(tl[e] + 1, minlength=p.C + 2).tolist() for e in range(p.J)]


def orbit_ids(p, g: Optional[vi.Grid] = None) -> np.ndarray:
    """Orbit of every state under host permutations: the occupancy with its
    digits sorted, re-encoded, plus the class block."""
    g = g or vi.grid(p)
    srt = np.sort(g.digits, axis=1)
    key = srt @ g.stride
    return (key[None, :] + np.arange(p.J)[:, None] * g.n_occ).reshape(-1)


def orbit_sum(p, x: np.ndarray, g: Optional[vi.Grid] = None) -> np.ndarray:
    """x summed over each orbit (indexed by the orbit's sorted-digit state)."""
    g = g or vi.grid(p)
    return np.bincount(orbit_ids(p, g), weights=np.asarray(x, dtype=np.float64),
                       minlength=p.J * g.n_occ)


# Orbit tables: one character per orbit (in increasing order of the orbit's
# representative state), 'a' + 1 + target load, '?' where the orbit holds an
# ambiguous state or its states disagree.
def orbit_table(p, tl: np.ndarray, amb, g: Optional[vi.Grid] = None) -> str:
    g = g or vi.grid(p)
    ids = orbit_ids(p, g)
    reps, inv = np.unique(ids, return_inverse=True)
    t = np.asarray(tl, dtype=np.int64)
    lo = np.full(reps.size, 127, dtype=np.int64)
    hi = np.full(reps.size, -127, dtype=np.int64)
    np.minimum.at(lo, inv, t)
    np.maximum.at(hi, inv, t)
    bad = lo != hi
    bad[np.unique(inv[np.asarray(amb, dtype=np.int64)])] = True
    chars = np.where(bad, ord("?"), ord("a") + 1 + lo).astype(np.uint8)
    return chars.tobytes().decode("ascii")


def expand_orbit_table(p, table: str, g: Optional[vi.Grid] = None) -> np.ndarray:
    """Target load of every state from an orbit table (-2 where it says '?')."""
    g = g or vi.grid(p)
    ids = orbit_ids(p, g)
    reps, inv = np.unique(ids, return_inverse=True)
    chars = np.frombuffer(table.encode("ascii"), dtype=np.uint8).astype(np.int64)
    if chars.size != reps.size:
        raise ValueError("orbit table does not match the instance")
    tl = np.where(chars == ord("?"), -2, chars - ord("a") - 1)
    return tl[inv]


def policy_from_target_load(p, tl: np.ndarray, g: Optional[vi.Grid] = None) -> np.ndarray:
    """The lowest-index host with the given occupancy (paid cloud for -1)."""
    g = g or vi.grid(p)
    tl = np.asarray(tl, dtype=np.int64).reshape(p.J, g.n_occ)
    pi = np.full((p.J, g.n_occ), p.K, dtype=np.int64)
    for e in range(p.J):
        hit = g.digits == tl[e][:, None]          # [n_occ, K]
        any_h = hit.any(axis=1)
        pi[e] = np.where(any_h & (tl[e] >= 0), np.argmax(hit, axis=1), p.K)
    return pi.reshape(-1).astype(np.uint8)
