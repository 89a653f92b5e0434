"""CPU oracle for CDEF (test infrastructure only; see cdef_oracle.h)."""
