"""Per-state definition of the uniformised occupancy MDP (oracle; test only).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The paper's MDP (Sec. V-B..V-G) is stated without rates; the readings taken
here are:

* State, Sec. V-B Eq. (10): s = (n_0..n_{K-1}, e).  n_k is the number of
  occupied VM units of vehicular cloud (host) k, 0 <= n_k <= C; the paper's
  "available VMs" M = C - n_k is implied by n and dropped; e is the class of
  the pending placement request (the next task to arrive).
  Index: occ(n) = sum_k n_k (C+1)^k (host 0 is the fastest digit) and
  s = occ(n) + e (C+1)^K (class slowest); N = J (C+1)^K.
* Actions, Sec. V-C Eq. (11): the paper's {picked VC, paid cloud} becomes
  a in {0..K-1} (place the request on host a, feasible iff n_a + size_e <= C)
  and a = K (send it to the paid traditional cloud; always feasible).
* Transitions, Sec. V-D Eqs. (12)-(13): placing a class-e task on host a adds
  size_e occupied units to that host (post-decision occupancy m = n + size_e
  1_a; m = n on reject).  Time is a continuous-time chain uniformised at
  Lam = sum_j lambda_j + K C mu + K nu.  One step is, with probability
    lambda_j / Lam      an arrival: the pending request is executed at n and
                        the next pending class is j -> (m, j);
    mu n_k / Lam        one occupied unit of host k is released -> (n - 1_k, e);
    nu / Lam            host k leaves and is replaced empty -> (n with n_k=0, e);
    the rest            nothing happens -> (n, e).
* Reward, Sec. V-E Eqs. (14)-(16): R(e, place) = r_e (the VC reward net of
  its cost), R(e, reject) = -c_e (the paid-cloud cost).  It accrues on the
  arrival branch only, so the expected one-step reward is P_arr R(e, a),
  P_arr = sum_j lambda_j / Lam.  The under-utilisation penalty of Eq. (16)
  (the paper's gamma_vc times the free VMs) is read as a cost
  ``idle_unit_cost`` u per free VM unit of every host, charged on every
  uniformised step: r(s, a) = P_arr R(e, a) - u (K C - sum_k n_k).  Every
  benchmark workload has u = 0.
* Bellman, Sec. V-G Eq. (18): with a discount gamma per uniformised step,
  Q(s,a) = r(s,a) + gamma sum_s' P(s'|s,a) V(s'), V(s) = max over feasible a.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Sequence, Tuple


def radix(p) -> int:
    return p.C + 1


def num_occupancies(p) -> int:
    return (p.C + 1) ** p.K


def num_states(p) -> int:
    return p.J * num_occupancies(p)


def num_actions(p) -> int:
    """K placements plus the paid-cloud action (Sec. V-C, Eq. (11))."""
    return p.K + 1


def encode(p, n: Sequence[int], e: int) -> int:
    """State index of (n, e) in the mixed-radix layout (Sec. V-B, Eq. (10))."""
    occ = 0
    mult = 1
    for k in range(p.K):
        occ += n[k] * mult
        mult *= p.C + 1
    return occ + e * mult


def decode(p, s: int) -> Tuple[Tuple[int, ...], int]:
    R = p.C + 1
    occ_count = R ** p.K
    e, occ = divmod(s, occ_count)
    n = []
    for _ in range(p.K):
        occ, d = divmod(occ, R)
        n.append(d)
    return tuple(n), e


def feasible_actions(p, s: int) -> List[int]:
    """Hosts with room for the pending task, then the paid cloud (always)."""
    n, e = decode(p, s)
    acts = [a for a in range(p.K) if n[a] + p.size[e] <= p.C]
    acts.append(p.K)
    return acts


def post_decision(p, n: Sequence[int], e: int, a: int) -> Tuple[int, ...]:
    """Occupancy after executing action a on the pending class-e task
    (Sec. V-D, Eq. (13): the chosen VC's occupied VMs grow by the task's need)."""
    if a == p.K:
        return tuple(n)
    m = list(n)
    m[a] += p.size[e]
    return tuple(m)


def uniformisation_rate(p, exact: bool = False):
    """Lam = sum_j lambda_j + K C mu + K nu (the largest total event rate)."""
    if exact:
        lam = [Fraction(x) for x in p.lam]
        return sum(lam) + p.K * p.C * Fraction(p.mu) + p.K * Fraction(p.nu)
    return sum(p.lam) + p.K * p.C * p.mu + p.K * p.nu


def reward(p, s: int, a: int, exact: bool = False):
    """Expected one-step reward P_arr * R(e, a) (Sec. V-E, Eqs. (14)-(16)),
    less the under-utilisation penalty of Eq. (16) on every free VM unit:
    idle_unit_cost * (K C - sum_k n_k)."""
    n, e = decode(p, s)
    F = Fraction if exact else float
    lam_tot = sum(F(x) for x in p.lam)
    Lam = uniformisation_rate(p, exact)
    R = F(p.reward[e]) if a < p.K else -F(p.reject_cost[e])
    free = p.K * p.C - sum(n)
    return lam_tot / Lam * R - F(p.idle_unit_cost) * free


def transitions(p, s: int, a: int, exact: bool = False) -> Dict[int, object]:
    """Successor distribution P(. | s, a) as {s': probability} (Sec. V-D).

    Written branch by branch as the uniformised chain defines it; repeated
    successors (a host reset that is already empty, the idle branch) are
    summed into one entry.
    """
    n, e = decode(p, s)
    if a not in feasible_actions(p, s):
        raise ValueError(f"action {a} infeasible in state {s}")
    F = Fraction if exact else float
    Lam = uniformisation_rate(p, exact)
    mu = F(p.mu)
    nu = F(p.nu)
    out: Dict[int, object] = {}

    def add(t, q):
        out[t] = out.get(t, 0) + q

    total = F(0)
    # arrival: the pending request is served by action a, next class j
    m = post_decision(p, n, e, a)
    for j in range(p.J):
        q = F(p.lam[j]) / Lam
        add(encode(p, m, j), q)
        total += q
    # one occupied unit of host k is released
    for k in range(p.K):
        if n[k] > 0:
            q = mu * n[k] / Lam
            dn = list(n)
            dn[k] -= 1
            add(encode(p, dn, e), q)
            total += q
    # host k leaves and is replaced by an empty one
    for k in range(p.K):
        q = nu / Lam
        rn = list(n)
        rn[k] = 0
        add(encode(p, rn, e), q)
        total += q
    # idle (uniformisation) branch
    add(s, 1 - total)
    return out


def bellman_backup(p, V: Sequence[float], s: int) -> Tuple[float, int, List[float]]:
    """One Bellman backup at state s (Eq. (18)): returns (max Q, lowest-index
    argmax, Q over feasible actions in action order).  V is any indexable of
    length N; arithmetic is Python float (FP64)."""
    qs = []
    acts = feasible_actions(p, s)
    for a in acts:
        acc = 0.0
        for t, q in transitions(p, s, a).items():
            acc += q * float(V[t])
        qs.append(reward(p, s, a) + p.gamma * acc)
    best = max(qs)
    arg = acts[qs.index(best)]
    return best, arg, qs


def empty_state_weights(p, exact: bool = False) -> List[object]:
    """Weights c_e = lambda_e / sum_j lambda_j of the states (0, e): the
    objective J = sum_e c_e V(0, e) is the expected discounted reward seen by
    a system that starts empty and waits for its first request."""
    F = Fraction if exact else float
    lam = [F(x) for x in p.lam]
    tot = sum(lam)
    return [x / tot for x in lam]
