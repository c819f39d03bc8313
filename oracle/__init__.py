"""FP64 CPU oracle of PARSDMM.  Test infrastructure only: the product path
never imports it."""
