"""FP64 CPU oracle for Batch-BFS search with the BCTS correction.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or run anything in this package; the product path
(the HIP library and its Python binding) never does.

It is a plain, slow, obviously correct evaluation of what the search computes:

* ``env``    -- the integer sprite environment (step, render, reward).
* ``qnet``   -- the Nature-DQN Q-network in FP64 (numpy), one stack at a time
                or a small batch of stacks.
* ``search`` -- the d-step value (Eq. 1) by recursive depth-first search,
                the depth-0/1 Bellman errors (Prop. 3.6), the penalty B
                (Eq. 6), the corrected root vector (Eq. 3) and its argmax
                (Eq. 4); plus enumeration of every tree node in the index
                order of Alg. 1 for bit-exact comparison of the expansion.
* ``gev``    -- the exact bias gap of Lemma 3.2 (Phi^-1 based) and its
                closed-form approximation of Lemma 3.4, for the exact-GEV
                correction mode.

It shares no code with the HIP path.  Inputs (environment tables, root
states, FP32 weights) come from ``paper_2107_01715_amd.workload``, which only
draws numbers.
"""
from . import env, qnet, search, gev  # noqa: F401
