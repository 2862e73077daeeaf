"""Encrypted clear-weight matrix products W.[x]_HE on packed RLWE ciphertexts for
AMD Instinct MI355X (gfx950): the server-side hot path of private LoRA
fine-tuning with homomorphic encryption (Frery et al., Sec. 4.3).

Importing the package loads nothing native; :mod:`paper_2505_07329_amd.rlwe`
loads the HIP library on first use and raises if it is missing.
"""
