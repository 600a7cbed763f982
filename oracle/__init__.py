"""Plain, slow CPU FP64 oracle for the PDEP chi0 path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs this
package; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the HIP library.

What it computes follows the paper's own definitions (Hartree units, e^2 = 1, Gamma
point, doubly occupied bands):

* plane-wave basis: all G with 1/2 |G|^2 <= E_cut (Sec. 2.1, plane-wave expansion);
* Kohn-Sham model Hamiltonian H = T + V_loc (Sec. 2, KS equation; local potential only);
* Sternheimer equation (H - e_v) P_c dpsi = -P_c dV psi_v (Sec. 2.3, Eq. stern);
* density response dn = sum over spin and bands of [dpsi* psi + c.c.] (Eq. deltani);
* chi0bar_ij = 4 pi <phi~_i | dn_j> with phi~ = phi/|G| (Eq. chiisamatrixinpdep,
  symmetrised form of Eq. symmoperator);
* sum-over-states (Adler-Wiser at omega = 0, q = 0 body, Eq. AdlerWiser) as a second,
  independent route to the same response;
* PDEP eigenpairs = lowest eigenpairs of chi0bar (Eq. eigendecompzerofreq);
* the reducible chibar = (1 - chi0bar)^-1 chi0bar (Eq. linearalgebrachichi0) and, as a
  second route, the self-consistent DFPT loop with the Hartree response (Eqs. LF and
  LFHartree, Fig. pdepscheme right panel); eps^-1 = 1 + chibar (Eq. epsilonandchi);
* the body, head and wings of chi0bar at imaginary frequencies (Eqs. AdlerWiser, finalF,
  finalU1, finalB) by sums over states, by resolvent solves and by deflated Lanczos
  chains (Sec. 2.4), and Lambda, Xi of Eq. Bfinal;
* G0W0 for occupied states: exchange, the correlation self-energy by contour deformation
  (Sec. 2.5) and the quasiparticle equation (Eqs. QPenergies, QPconZ).

Modules:
  planewave  -- sphere, grid, naive DFT, dense H
  response   -- ground state, direct and sum-over-states Sternheimer, dn, chi0bar, PDEP
  matfree    -- matrix-free FFT + CG version of the same chain (used for CPU timing and
                sampled checks at sizes where dense matrices do not fit)
  lanczos    -- body of chi0bar at imaginary frequencies, sums over states and chains
  headwings  -- head and wings at q -> 0, the Brillouin-zone Coulomb integral, Eq. Bfinal
  gw         -- Sigma_X, Sigma_C by contour deformation, QP energies
"""
