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

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, textbook identities, brute
force or invariants; none is marked "parity unpinned" except where the
function header says so.
"""
