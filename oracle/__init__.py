"""CPU oracle for the attestation check -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it, and it never imports them.
"""
from .oracle import (  # noqa: F401
    build,
    constants,
    sha256,
    sha256_compress,
    sha256_iv,
    hmac_sha256,
    hmac_midstates,
    hkdf_sha256,
    derive_keys,
    derive_keys_multi,
    verify_batch,
    verify_batch_rev,
    verify_attest,
    poh_verify,
    merkle_roots,
)
