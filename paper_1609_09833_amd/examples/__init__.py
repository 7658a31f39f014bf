"""Clients of libabp.so's C-ABI that are not part of the library: a plain C
client (abp_c_client.c) and an open-loop load generator for the serving loop
(abp_serve_driver.cpp, bound by serve_driver.py)."""
