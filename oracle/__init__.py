"""CPU oracle for data-race freedom of memory access protocols.

Test infrastructure: only the tests, the smoke check and the bench's CPU
baseline use it.  It shares no code with the HIP path.
"""
