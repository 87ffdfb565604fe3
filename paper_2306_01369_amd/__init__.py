"""MI355X-native granular contact step (spatial-hash detection + projected Jacobi).

Importing the package loads nothing native; ``paper_2306_01369_amd.gg``
binds the C-ABI library ``libgg.so``.
"""
__all__ = ["scenes", "gg"]
