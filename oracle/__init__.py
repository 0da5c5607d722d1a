"""Plain FP64 CPU oracle for the tensor-network Metropolis-Hastings hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import anything here.  The
product path (the HIP library and its Python binding) never imports, calls or
links this package, and this package never imports the product.

Every function follows a passage of the paper (arXiv:2104.13264, "Collective
Monte Carlo updates through tensor network renormalization") and cites it by
section / equation / algorithm.  The arithmetic is NumPy float64 with library
QR/SVD/matmul as the only black boxes; there is no blocking, fusion or
reordering beyond what the cited passages state.

Modules
    philox   counter-based RNG (Philox4x32-10, Salmon et al., SC'11)
    ising    Eq. (ising) energy, App. A bond matrices W and their split
    exact    brute-force enumeration, exact row transfer matrix, Onsager
    bmps     App. A boundary-MPS contraction (MPO on MPS, successive SVD)
    sampler  Sec. 2 sequential (Bayes chain-rule) sampler, Eqs. (bayes),
             (pi-approx), App. A Eq. (proba-ratio-apx); sample and eval modes
    mh       Algorithm 1 (TNMH Markov chain) with Eqs. (mh-acc), (tns-prior)
    stats    Eqs. (cauto), (c-auto-int): autocorrelation, tau_int
    grad     derivative of ln Z~ with frozen truncation isometries
    metropolis  single-spin-flip sweeps interleaved with TNMH steps
    periodic periodic boundaries by alternately frozen lines (Sec.
             "Arbitrary boundary conditions")
    potts    q-state Potts models, general local dimension d (App. A
             Eqs. pf_bond_description, tensor-general; Sec. 2)

Parity status: every function is pinned by the CPU tests (tests/test_oracle_*.py)
against brute force, exact transfer matrices, closed forms, invariants or an
independent library run, except where a module header says "parity unpinned".
"""
