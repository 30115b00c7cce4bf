"""MI355X ensemble MHD time step (decoupled Elsasser scheme, shared matrix for J members).

The numerical work lives in the HIP library ``libmhd_ens.so`` (sources in
``csrc/``, C ABI in ``include/mhd_ens.h``); ``_lib`` is its ctypes binding and
``ensemble`` a small driver that keeps the state in device memory.
"""
__all__ = ["_lib", "ensemble"]
