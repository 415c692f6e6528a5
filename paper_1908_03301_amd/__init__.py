"""MI355X-native solver for steady flow through random resistor / pore networks.

The solve runs in the HIP library ``librn.so`` (built from ``csrc/``) behind a
C ABI declared in ``include/rn.h``; ``binding`` marshals Python arguments to
it. ``inputs`` generates seeded synthetic networks. Importing the package
loads nothing; the library is loaded on first use of the binding.
"""
__all__ = ["inputs", "binding"]
