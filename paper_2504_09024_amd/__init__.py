"""MI355X-native coupled central-moment lattice Boltzmann step for
interface-bound surfactant transport (arXiv 2504.09024).

The step runs in hand-written HIP kernels behind the C ABI declared in
``include/cmlb.h``; ``paper_2504_09024_amd.cmlb`` is the thin ctypes binding
and ``paper_2504_09024_amd.workloads`` builds synthetic inputs.  Importing the
package loads nothing native; the binding loads ``libcmlb.so`` on first use
and raises if it is missing.
"""
__all__ = ["cmlb", "workloads"]
