"""MI355X-native Shared Response Model EM sweep (arXiv 1608.04647, Sec. II).

``synth`` draws seeded inputs; ``srm`` binds the HIP C-ABI library
(``libsrm.so``).  Importing the package loads nothing; ``srm`` raises at
import if the library has not been built.
"""
__all__ = ["synth", "srm"]
