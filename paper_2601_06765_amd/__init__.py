"""MI355X (gfx950) F4 reduction step over F_p: symbolic preprocessing
(sorted monomial dictionary, two-pass CSR assembly) and elimination mod p,
behind the C-ABI of include/f4.h.  `f4` is the ctypes binding of libf4.so."""

__all__ = ["f4"]
