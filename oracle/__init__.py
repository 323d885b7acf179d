"""Plain FP64 CPU oracle of the RCB tree method (Gafton & Rosswog 2011).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg. The product path (the HIP library and its Python
binding) never imports, links or runs anything in this package.
"""
