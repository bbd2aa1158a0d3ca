"""Monolithic AMG (defect correction, Vanka / DLSC) Stokes solve phase on MI355X."""
