"""Plain, slow FP64 CPU oracle for the occupancy-MDP value-iteration path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls anything here.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

Modules
-------
model   per-state definitions: state encoding, feasible actions, transition
        list and immediate reward, written one state at a time (Sec. V-B..V-E).
vi      whole-state-space FP64 Jacobi value iteration, greedy extraction,
        fixed-policy evaluation and the fast greedy heuristic (Eq. (18),
        Alg. 3, Alg. 2), vectorised with NumPy index arithmetic.
exact   exact rational (``fractions.Fraction``) solves and brute force over
        all deterministic policies for tiny instances.
grad    gradient of the expected discounted reward from the empty system
        with respect to (lambda_j, mu, nu, r_j): dense autograd, sparse
        adjoint and central finite differences.
bsdi    block-asynchronous value iteration on occupancy tiles (Alg. 4).
pi      policy iteration with a near-tie guard (Alg. 3 step 4 repeated).
static_bot  the fast greedy heuristic (Alg. 2) on a static set of bags of
        tasks, the cloud-wide reward of a placement (Eqs. (14)-(16)) and the
        best placement by search (Sec. VII example).

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, textbook identities, brute
force or invariants; none is marked "parity unpinned" except where the
function header says so.
"""
