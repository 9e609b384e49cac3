"""spic: MI355X-native implicit particle-in-cell mover and moment gathering.

Importing the package loads nothing native; the HIP library is opened on
first use of :mod:`paper_2008_04397_amd.spic`.
"""
