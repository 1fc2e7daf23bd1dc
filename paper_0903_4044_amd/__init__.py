"""MI355X-native BGK discrete-velocity stepper (hand-written HIP for gfx950).

Importing the package loads nothing; ``paper_0903_4044_amd.binding`` loads the
HIP library ``libbgk.so`` and fails loudly when it is missing.
"""
