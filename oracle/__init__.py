"""FP64 CPU oracle of the random batch Ewald method (arXiv:2110.14362).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path (librbe.so and its
binding) never does, and shares no code with it.

Modules
    philox     Philox4x64-10 counter-based generator (SC'11 definition)
    sampler    per-axis discrete-Gaussian tables and the batch draw (sections 4.2-4.3)
    ewald      classical Ewald energy, forces and virial, general cell (section 4.1, app. C)
    rbe        random batch estimators on an explicit batch; Prop. 1 variances (section 4.2, 4.4)
    realspace  nearest-image real-space erfc sum with a cutoff (section 4.2)

Pinned by the `-m "not gpu"` tests against closed forms, library routines and
finite differences; see each module's docstring for the passage it follows.
"""
