"""CPU oracle for PUMP's exploration hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 numpy implementation of what the planner computes, written
from the paper (Ichter, Schmerling, Agha-mohammadi, Pavone, "Real-Time
Stochastic Kinodynamic Motion Planning via Multiobjective Search on GPUs",
arXiv 1607.06886).  It exists to check the HIP implementation: only the test
suite, the package smoke check and the benchmark's CPU-baseline leg may import
or run it.  The product path never routes through it, and it shares no code,
tables or constants with the HIP library; both sides take their inputs from the
seeded generators in ``paper_1607_06886_amd.scenes``.

Modules
  dynamics  -- eq. (1)-(2) discretisation, the tracking controller of Sec. II,
               the particle deviation table (Sec. III-B particles).
  steer     -- Cost(u, v): the optimal double-integrator connection (Sec. IV
               primitives, cost c of Sec. II).
  graph     -- BuildGraph (Alg. 3) with Near and an exact Collision(u, v).
  explore   -- Explore (Alg. 4) with the particle CP estimate and
               RemoveDominated (Sec. IV primitives).
  select    -- MC(p) and PlanSelection (Alg. 5).
  pump      -- PUMP main (Alg. 2) and the parameters the paper leaves open.

Every function names the passage it follows.  Points where the paper is silent
or ambiguous are resolved by the readings listed in the repository's design
notes; each is restated where it is used.
"""
