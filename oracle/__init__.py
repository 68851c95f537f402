"""CPU FP64 oracle for the multi-component pseudo-potential lattice Boltzmann model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP path (no common kernels, tables, helpers or constant generators).

The oracle is written for a reader who holds the paper (Peng, Ayala & Ayala,
"A thermodynamically consistent pseudo-potential lattice Boltzmann model for
multi-component, multiphase, partially miscible mixtures", arXiv 1909.12390):
every function cites the section / equation it follows and is a plain,
unblocked, unfused transcription in float64 NumPy.

Modules
-------
thermo   Peng-Robinson mixture thermodynamics (Sec. 3.2): EOS, cubic in Z,
         fugacity coefficients, Gibbs root choice, flash, bubble/dew points,
         Maxwell construction, volatility coefficients gamma (Sec. 3.1).
lattice  D2Q9 / D3Q19 velocity sets and the orthogonal MRT moment bases.
lbm      One time step of the model (Sec. 2.1 LBE, Sec. 3.1/3.3 forces,
         Sec. 3.4 order of operations) plus moments and conservation sums.

Parity status per function is listed in each module header.
"""
