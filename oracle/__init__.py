"""FP64 CPU oracle for stochastic matrix-free equilibration (Diamond & Boyd).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct CPU
implementation of what the GPU library computes.  Only the test suite, the smoke
check of the package entry module and the CPU-baseline leg of the benchmark may
import it.  The GPU library never imports, links or calls anything here, and this
package imports nothing from the GPU library: the two share no code.

Contents
  signs      -- the probe sign contract (Philox4x64-10 bit stream), via numpy.
  algorithm1 -- projected stochastic gradient (Algorithm 1, Section 3.2), with
                k probes per step, warm starts and a step offset.
  theory     -- objective, exact gradient, estimator, Sinkhorn-Knopp (Section 2.1),
                Lambert-W block minimisation (Section 2.3), Newton (Section 4),
                Phi and the condition-number bound (Section 2.2).
  metrics    -- RMS equilibration error (Section 4), relative optimality gap.
  lsqr       -- LSQR (Paige & Saunders) on the scaled system of Section 5.1.
  variants   -- Section 6: symmetric equilibration (Algorithm 2), varying row and
                column norms, block equilibration.
  ccp        -- Chambolle-Cremers-Pock on the Lasso, with and without equilibration
                (Section 5.2).

Every function is pinned by a test in tests/test_oracle_*.py against something
other than itself (closed forms, enumeration, library routines, theorems).
"""
