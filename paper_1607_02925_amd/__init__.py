"""MI355X (gfx950) implementation of shift-and-invert block power iteration
with oversampling and SVRG inner solves, behind the C ABI in include/lowrank.h.
"""
