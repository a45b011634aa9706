"""FP64 CPU oracle of the FastVPINNs loss (test infrastructure only; the library never imports it)."""
