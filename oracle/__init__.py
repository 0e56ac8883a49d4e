"""Plain FP64 CPU oracle for the separable planewave Coulomb scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, link or call anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code, header, table or constant generator with the GPU path.

What it computes (Pederson, "Practical and Rigorous Reduction of the
Many-Electron Quantum Mechanical Coulomb Problem to O(N^{2/3}) Storage"):

* basis    -- planewaves exp(2 pi i n.r / L) with |n|^2 <= n2max (Sec. II, the
              cutoff on |I|; Sec. III shell closings), canonical order.
* mesh     -- Gauss-Legendre nodes on the Laplace variable split at the cutoff,
              with the t = 1/sqrt(alpha) map on the tail (Eqs. 10-14), and the
              geometric "Mesh 2" sub-intervals (Sec. III, Table I); "Mesh 3"
              integrates the same pieces in sqrt(beta) and the tail with a
              rule for polynomials in t^2 (Sec. II, after Eq. 14).
* tables   -- the 1-D integral of Eq. 8 for planewave factors, one table per
              quadrature node indexed by the two wavevector differences;
              for a rectangular box one such table per direction, at the
              node scaled by that direction's side (box_tables).
* sums     -- the node sum of Eq. 14 (reconstruction of <ij|kl>) and the
              uniform-electron-gas Hartree / exchange pair sums of Sec. III,
              in plain C with Neumaier-compensated FP64 accumulation.
* gauss    -- the same scheme for a separable s-type Gaussian basis (Sec. II):
              pair products, the closed-form 1-D factor, screened pairs, and
              the node sum over the three direction factors.
* exchange_hist -- an independent route to the exchange energy through the
              histogram of wavevector differences (cross-check only).

Functions whose result is not pinned by a test against the paper or against
the mathematics say "parity unpinned" in their docstring; at present there
are none.
"""
from .basis import enumerate_basis, shell_counts
from .mesh import gauss_legendre, mesh1, mesh2, mesh3, default_mesh
from .tables import primitives, tau_table, tau_diag, tau00_closed_form, box_tables
from .sums import reconstruct, energies
from .exchange_hist import diff_histogram, exchange_from_histogram
from .gauss import gauss_pairs, pair_params, gauss_G, gauss_tau, gauss_decode, gauss_reconstruct
from .physics import e_ks, k_cube

__all__ = [
    "enumerate_basis", "shell_counts", "gauss_legendre", "mesh1", "mesh2", "mesh3",
    "default_mesh", "primitives", "tau_table", "tau_diag", "tau00_closed_form", "box_tables",
    "reconstruct", "energies", "diff_histogram",
    "exchange_from_histogram", "e_ks", "k_cube", "gauss_pairs", "pair_params", "gauss_G",
    "gauss_tau", "gauss_decode", "gauss_reconstruct",
]
