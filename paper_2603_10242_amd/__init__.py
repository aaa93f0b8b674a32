"""MI355X-native batched verification of HMAC-SHA256 attestations under
HKDF-SHA256 derived keys (the ACE Runtime's AttestCheck, Alg. 1 Phase 1a).

Import ``paper_2603_10242_amd.ace`` for the binding over ``libace.so``;
``paper_2603_10242_amd.workload`` draws seeded synthetic batches.  Importing
the package itself loads nothing.
"""
