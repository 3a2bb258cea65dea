"""MI355X (gfx950) implementation of count-sketch LSH indexing.

Importing the package loads nothing native; ``paper_2503_06737_amd.lsh``
loads the HIP library ``liblsh.so`` on first use and raises if it is missing.
"""
